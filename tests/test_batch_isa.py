"""CPU-only check of the batch transform kernel's gfx950 code: it reads its
buffer addresses from pass records in device memory, and must still access
the data and twiddles with global (not flat) loads and stores, as the plain
pass kernel does with addresses passed as kernel arguments.  A flat access
also counts on the LDS wait counter, so each LDS wait of a round would wait
for the HBM loads in flight too."""
import importlib.util
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_07535_amd", "csrc")

SRC = """#include "ntt_impl.hpp"
namespace moma {
template __global__ void ntt_batch_kernel<2, 1, false, false, false>(const NttPassArgs*, const NttC<2, false>*,
                                                                     const uint2*, u32);
template __global__ void ntt_batch_kernel<4, 2, true, false, false>(const NttPassArgs*, const NttC<4, false>*,
                                                                    const uint2*, u32);
template __global__ void ntt_pass_kernel<4, 2, true, false, kArithLazy>(NttPassArgs, NttC<4>);
}
"""


def _kernels(asm: str) -> dict:
    """kernel symbol -> its instruction mnemonics"""
    out = {}
    lines = asm.splitlines()
    starts = [i for i, l in enumerate(lines) if re.match(r"^_Z\S*:", l)] + [len(lines)]
    for a, b in zip(starts, starts[1:]):
        name = lines[a].split(":")[0]
        out[name] = [l.split()[0] for l in lines[a + 1:b]
                     if l.startswith("\t") and not l.strip().startswith((".", ";"))]
    return out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc is not available")
def test_batch_kernels_use_global_memory_instructions(tmp_path):
    spec = importlib.util.spec_from_file_location("moma_build_script", os.path.join(ROOT, "paper_2501_07535_amd", "build.py"))
    build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(build)
    src = tmp_path / "batch_isa.hip"
    src.write_text(SRC)
    asm = tmp_path / "batch_isa.s"
    r = subprocess.run(["hipcc", *build.FLAGS, "--cuda-device-only", "-S", f"-I{CSRC}", f"-I{ROOT}/include",
                        str(src), "-o", str(asm)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    ks = _kernels(asm.read_text())
    batch = {k: v for k, v in ks.items() if "ntt_batch_kernel" in k}
    plain = {k: v for k, v in ks.items() if "ntt_pass_kernel" in k}
    assert len(batch) == 2 and len(plain) == 1
    for name, ins in batch.items():
        flat = [m for m in ins if m.startswith("flat_")]
        glob = [m for m in ins if m.startswith(("global_load", "global_store"))]
        assert not flat, (name, sorted(set(flat)))
        assert glob, name
    # the multiplying variant at 4 limbs: the same memory instructions as the plain kernel
    mem = lambda ins: sorted(m for m in ins if m.startswith(("global_", "flat_", "buffer_")))
    b4 = next(v for k, v in batch.items() if "Li4ELi2E" in k)
    p4 = next(iter(plain.values()))
    assert mem(b4) == mem(p4)
