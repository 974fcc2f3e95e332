"""CPU-only memory and undefined-behaviour checks of the host code: the oracle
(plain C) and the library's host big integers (hostbig.hpp), each built with
AddressSanitizer and UBSan (any report is fatal) and run on their own checks.

* The oracle's pins (tests/test_oracle_*.py) run once more, in a child
  process, against a sanitized build of oracle/moma_oracle.c.
* hostbig.hpp is driven through a small test program on random and edge
  operands; every result is compared with Python integers.
"""
import os
import random
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _asan_runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


needs_gcc = pytest.mark.skipif(shutil.which("gcc") is None or _asan_runtime() is None,
                               reason="gcc with the AddressSanitizer runtime is not available")


@needs_gcc
def test_oracle_pins_under_address_and_ub_sanitizers(tmp_path):
    import oracle
    lib = oracle.build(out=str(tmp_path / "libmoma_oracle_san.so"), flags=SAN)
    env = dict(os.environ)
    env.update({"MOMA_ORACLE_LIB": lib, "LD_PRELOAD": _asan_runtime(),
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1",
                "OMP_NUM_THREADS": "4"})
    tests = sorted(os.path.join(ROOT, "tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail


def _cases(seed=7, count=150):
    rng = random.Random(seed)
    edge = [0, 1, 2, (1 << 32) - 1, 1 << 32, (1 << 64) - 1, (1 << 1024) - 1, (1 << 1020) + 1]
    out = []
    for k in range(count):
        bits = rng.choice([1, 31, 32, 33, 63, 64, 65, 127, 256, 511, 1024, 2048])
        a = rng.getrandbits(bits) if k % 9 else rng.choice(edge)
        b = rng.getrandbits(rng.choice([1, 32, 64, 200, 1024])) if k % 7 else rng.choice(edge)
        m = rng.getrandbits(rng.choice([33, 64, 252, 1020, 1024])) | 1
        out.append(("add", a, b))
        out.append(("sub", max(a, b), min(a, b)))
        out.append(("mul", a, b))
        out.append(("shl", a, rng.randrange(0, 100)))
        out.append(("shr", a, rng.randrange(0, 1100)))
        if b:
            out.append(("divmod", a, b))
        if m > 1:
            out.append(("mulmod", a % m, b % m, m))
            out.append(("powmod", a, rng.getrandbits(rng.choice([1, 8, 64, 300])), m))
        out.append(("ninv", a | 1))
    return out


def _expect(c):
    op = c[0]
    if op == "add":
        return hex(c[1] + c[2])
    if op == "sub":
        return hex(c[1] - c[2])
    if op == "mul":
        return hex(c[1] * c[2])
    if op == "shl":
        return hex(c[1] << c[2])
    if op == "shr":
        return hex(c[1] >> c[2])
    if op == "divmod":
        return f"{hex(c[1] // c[2])} {hex(c[1] % c[2])}"
    if op == "mulmod":
        return hex(c[1] * c[2] % c[3])
    if op == "powmod":
        return hex(pow(c[1], c[2], c[3]))
    return hex((-pow(c[1] & 0xFFFFFFFF, -1, 1 << 32)) % (1 << 32))


@needs_gcc
@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not available")
def test_host_big_integers_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "hostbig_driver")
    src = os.path.join(ROOT, "tests", "sanitize", "hostbig_driver.cpp")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-o", exe, src])
    cases = _cases()
    lines = []
    for c in cases:
        # operands in hexadecimal; a shift count in decimal
        args = [str(v) if (i == 1 and c[0] in ("shl", "shr")) else hex(v) for i, v in enumerate(c[1:])]
        lines.append(" ".join([c[0], *args]))
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                                UBSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    got = r.stdout.splitlines()
    assert len(got) == len(cases)
    for c, g in zip(cases, got):
        assert g == _expect(c), (c[0], [hex(v) for v in c[1:]], g)
