"""Benchmark: 256-bit forward NTT, n = 2^20, on one MI355X.

One step is one forward transform y = NTT(x) (Eq. (ntt)) of 2^20 residues mod a
seeded 252-bit prime q = c*2^32 + 1 stored as 8 limb planes, input resident in
HBM, output to a second resident buffer.  The value is butterflies per second,
B(n) = (n/2) log2 n butterflies per step (the paper's count, Section 5.3).

Printed: one JSON line with the contract fields plus
  roofline:     the transform kernel against the integer-VALU peak,
  cpu_baseline: the oracle's transform timed on the host cores,
  extras:       inverse transform time, the paper's ns/butterfly, checks.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import moma_inputs as mi  # noqa: E402

# MI355X integer VALU peak: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
# (full-rate 32-bit lane operations, wave64).  How fast the instructions of a
# modular multiply actually issue relative to that is measured by the library's
# own probes (moma_measure_peaks) in every run.
PEAK_INT_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12
VALU_SIMDS, CLOCK_HZ = 256 * 4, 2.4e9


def word_products(L: int) -> int:
    """P(L): 32x32-bit word products of one L-limb Montgomery multiply
    (2L^2 + L: the L x L product and the reduction's L x L + L)."""
    return 2 * L * L + L


def issue_costs(rates: dict) -> tuple[float, float]:
    """Cost of one word product with its carry step (a v_mad_u64_u32 whose
    carry-out feeds a v_addc_co_u32) and of one add-class op (an add or
    subtract with carry), in peak lane-ops: the time the instructions take at
    their measured issue rates, times PEAK_INT_OPS.  Work priced this way and
    divided by PEAK_INT_OPS is the time the work takes at the measured rates,
    so achieved / peak is that time over the measured time."""
    return 2.0 * PEAK_INT_OPS / rates["mad_addc_u32"], PEAK_INT_OPS / rates["add_co_addc_u32"]


def multiply_forms(L: int, rates: dict) -> dict:
    """Work of one L-limb Montgomery multiply in peak lane-ops, in its two
    gfx950 forms.  Word form: P(L) 32-bit word products, each a v_mad_u64_u32
    plus the v_addc_co_u32 that takes its carry.  Digit form (the same
    multiply on D digits of b bits, b = 29 up to 28 limbs, else 28, D =
    ceil((32L - 2) / b)): 2D^2 digit products, each one v_mad_u64_u32 and no
    carry step (a column of them stays below 2^64), one v_mul_lo_u32 per
    reduction digit, and two add-class ops per column (shift and mask)."""
    cm, ca = issue_costs(rates)
    b = 29 if L <= 28 else 28
    D = -(-(32 * L - 2) // b)
    word = word_products(L) * cm
    digit = (2 * D * D * PEAK_INT_OPS / rates["mad_u64_u32"] + D * PEAK_INT_OPS / rates["mul_lo_u32"]
             + 2 * (2 * D - 1) * ca)
    return {"word": word, "digit": digit, "digits": D}


def butterfly_slots(L: int, rates: dict) -> float:
    """Work of one butterfly under the op model, in peak lane-ops: one L-limb
    Montgomery multiply in the cheaper of its two forms (multiply_forms) plus
    a modular add and a modular subtract (3L add-class ops each: the chain,
    the trial subtraction, the select)."""
    cm, ca = issue_costs(rates)
    f = multiply_forms(L, rates)
    return min(f["word"], f["digit"]) + 6 * L * ca


def blas_slots(op: str, L: int, rates: dict, karatsuba: bool = False) -> float:
    """Work per element of one BLAS op under the same op model, in peak lane-ops.  vmul
    (Barrett): two full L x L products (3 ceil(L/2)^2 word products each by
    Karatsuba, else L^2) and the low half of r2 * q (L(L+1)/2), plus 3L for the
    subtraction and correction; axpy: a Montgomery multiply by alpha (P(L))
    with its correction (2L) and a modular add (3L); vadd/vsub: 3L."""
    cm, ca = issue_costs(rates)
    if op in ("vadd", "vsub"):
        return 3 * L * ca
    if op == "vmul":
        h, g = (L + 1) // 2, L // 2
        full = 2 * h * h + g * g if karatsuba else L * L
        return (2 * full + L * (L + 1) // 2) * cm + 3 * L * ca
    return word_products(L) * cm + 5 * L * ca


def host_cpu() -> dict:
    """CPU model and core counts of the host the oracle baseline ran on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--lam", type=int, default=256, help="bit-width class")
    ap.add_argument("--logn", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--batch-jobs", type=int, default=4096)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--no-tune", action="store_true", help="time the default schedule without autotuning")
    ap.add_argument("--settle", type=float, default=0.25,
                    help="seconds of untimed transforms before the autotuner, before the warm-up steps and before "
                         "timing each steady-state batch (the clock's ramp)")
    ap.add_argument("--schedule", default=None,
                    help="tile_log,col_log,threads,radix_log[,mul_variant]: use this launch shape instead of "
                         "autotuning")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline line, print one JSON line per size of the transform sweep "
                         "(2^16..2^24 at 256 bits, 2^20 at 128/384/1024 bits, and 2^20 with full-width "
                         "256- and 1024-bit moduli)")
    ap.add_argument("--forward-only", action="store_true",
                    help="time only the headline forward transform (no default-schedule, inverse or cyclic-product "
                         "timing): every transform kernel launched is a headline pass, for counter collection")
    ap.add_argument("--blas", action="store_true",
                    help="instead of the headline line, print one JSON line per modular BLAS op and width "
                         "(vadd/vsub/vmul/axpy at n=2^24, 256/384/768 bits)")
    ap.add_argument("--blas-logn", type=int, default=24)
    ap.add_argument("--mulalg", action="store_true",
                    help="instead of the headline line, compare the butterfly's schoolbook and Karatsuba word "
                         "products (Eq. (mulk)) at n=2^12 for 128, 256, 384 and 768 bits")
    ap.add_argument("--peaks", action="store_true",
                    help="instead of the headline line, print the measured issue rates and HBM bandwidths that "
                         "price the roofline")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def sweep(args):
    """One line per sweep size: autotuned single-call time, steady state over k, and
    the oracle's sampled outputs."""
    import torch

    import oracle
    import paper_2501_07535_amd as moma
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rates = moma.measure_peaks()
    # (class, log2 n, modulus bits): the paper's lam - 4 bit moduli, then full-width
    # moduli (bitlen q = lam, no headroom) at 256 and 1024 bits
    shapes = [(256, l, None) for l in range(16, 25)] + [(128, 20, None), (384, 20, None), (1024, 20, None),
                                                         (256, 20, 256), (1024, 20, 1024)]
    for lam, logn, bits in shapes:
        f = mi.find_prime(lam, 0, bits=bits) if bits else mi.find_prime(lam, 0)
        L, n, q = f.limbs, 1 << logn, f.q
        w = f.root(n)
        x = mi.residues(f, n, L, 2, logn)
        dx = torch.from_numpy(mi.to_planar(x).view(np.int32)).to(dev)
        dy = torch.empty_like(dx)
        moma.ntt_prepare(q, w, n, L)
        _settle_fwd(moma, torch, dx, dy, q, w, args.settle)
        tuned = moma.ntt_tune(q, w, n, L, reps=3, warmup=1)
        steps = max(3, min(50, int(2e5 / max(tuned["best_us"], 1.0))))
        _settle_fwd(moma, torch, dx, dy, q, w, args.settle)
        us = _time_fwd(moma, torch, stream, dx, dy, q, w, 2, steps)
        ks = np.array([0, 1, n - 1], dtype=np.int64)
        got = mi.from_planar(dy[:, torch.from_numpy(ks).to(dev)].cpu().numpy().view(np.uint32))
        ok = bool((got == oracle.ntt_direct(q, L, w, x, ks)).all())
        # batches of up to 64 transforms, as far as 16 GiB of inputs and outputs allow
        per = 2 * n * 4 * L
        kmax = max(1, min(64, (16 << 30) // per))
        kmax = 1 << (kmax.bit_length() - 1)
        st = steady_state(moma, torch, stream, dx, q, w, n, L, logn,
                          ks=tuple(sorted({k for k in (1, 4, 16, 64) if k <= kmax} | {kmax})), settle=args.settle)
        B = n // 2 * logn
        print(json.dumps({"lambda": lam, "limbs": L, "q_bits": q.bit_length(), "full_width": bool(bits),
                          "log2_n": logn, "fwd_us": round(us, 2),
                          "gbutterfly_s": round(B / us / 1e3, 3), "steady_state": st,
                          "schedule": list(moma.ntt_get_schedule(q, w, n, L)),
                          "alu_frac": round(butterfly_slots(L, rates) * B / (us * 1e-6) / PEAK_INT_OPS, 4),
                          "sampled_vs_oracle": ok}), flush=True)
        del dx, dy
        moma.shutdown()


def blas(args):
    """One line per (op, width): time per call with inputs resident, achieved
    GB/s and integer op rate, the binding roofline, and outputs checked at
    sampled indices against the oracle."""
    import torch

    import oracle
    import paper_2501_07535_amd as moma
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    n = 1 << args.blas_logn
    rates = moma.measure_peaks()
    idx = np.array([0, 1, n // 3, n // 2 + 7, n - 2, n - 1], dtype=np.int64)
    for lam in (256, 384, 768):
        f = mi.find_prime(lam, 0)
        L, q = f.limbs, f.q
        da = torch.from_numpy(mi.to_planar(mi.residues(f, n, L, 1, 1)).view(np.int32)).to(dev)
        db = torch.from_numpy(mi.to_planar(mi.residues(f, n, L, 1, 2)).view(np.int32)).to(dev)
        dc = torch.empty_like(da)
        alpha = mi.scalar_residue(f, 1, 3)
        calls = {"vadd": lambda: moma.vadd(da, db, q, out=dc), "vsub": lambda: moma.vsub(da, db, q, out=dc),
                 "vmul": lambda: moma.vmul(da, db, q, out=dc), "axpy": lambda: moma.axpy(alpha, da, db, q, out=dc)}
        # vmul: the autotuner picks schoolbook or Karatsuba products for this width
        tuned = moma.vmul_tune(q, L, n, reps=5)
        for op, fn in calls.items():
            # warm up for at least ~0.2 s of this op: the clock settles to the
            # op's own power draw (a few calls right after a memory-bound op
            # time the multiply-heavy ones up to 15% slow)
            t0 = time.time()
            k = 0
            while k < args.warmup or time.time() - t0 < 0.2:
                fn()
                k += 1
                if k % 16 == 0:
                    torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(args.steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / args.steps
            sel = torch.from_numpy(idx).to(dev)
            a = mi.from_planar(da[:, sel].cpu().numpy().view(np.uint32))
            bb = mi.from_planar(db[:, sel].cpu().numpy().view(np.uint32))
            got = mi.from_planar(dc[:, sel].cpu().numpy().view(np.uint32))
            want = {"vadd": lambda: oracle.vadd(q, L, a, bb), "vsub": lambda: oracle.vsub(q, L, a, bb),
                    "vmul": lambda: oracle.vmul(q, L, a, bb), "axpy": lambda: oracle.axpy(q, L, alpha, a, bb)}[op]()
            byt = 3 * n * 4 * L
            slots = blas_slots(op, L, rates, karatsuba=(op == "vmul" and tuned["chosen"] == moma.VMUL_KARATSUBA)) * n
            t_hbm, t_alu = byt / PEAK_HBM, slots / PEAK_INT_OPS
            bound = "hbm" if t_hbm >= t_alu else "alu"
            print(json.dumps({"op": op, "lambda": lam, "limbs": L, "log2_n": args.blas_logn, "us": round(us, 2),
                              "GB_s": round(byt / us / 1e3, 1), "Tops_s": round(slots / us / 1e6, 3),
                              "bound": bound, "roofline_us": round(max(t_hbm, t_alu) * 1e6, 2),
                              "frac": round(max(t_hbm, t_alu) * 1e6 / us, 4),
                              "hbm_frac": round(t_hbm * 1e6 / us, 4), "alu_frac": round(t_alu * 1e6 / us, 4),
                              "vmul_variants": tuned if op == "vmul" else None,
                              "sampled_vs_oracle": bool((got == want).all())}), flush=True)
        del da, db, dc
        torch.cuda.empty_cache()


def mulalg(args):
    """The butterfly's word-product form (Eq. (mulk)) at n = 2^12: for each width
    the autotuner times every launch shape with the schoolbook and (radix-2
    shapes) the Karatsuba digit product; the best of each form is re-timed,
    then both forms on the best Karatsuba shape, with outputs checked against
    the oracle's transform."""
    import torch

    import oracle
    import paper_2501_07535_amd as moma
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    logn = 12
    n = 1 << logn
    for lam in (128, 256, 384, 768):
        f = mi.find_prime(lam, 0)
        L, q = f.limbs, f.q
        w = f.root(n)
        x = mi.residues(f, n, L, 2, logn)
        want = oracle.ntt_radix2(q, L, w, x)
        dx = torch.from_numpy(mi.to_planar(x).view(np.int32)).to(dev)
        dy = torch.empty_like(dx)
        moma.tune_db_clear()
        moma.ntt_tune(q, w, n, L, reps=3, warmup=1)
        rows = moma.tune_db_rows()

        def best(pred):
            r = min((r for r in rows if pred(r["sched"])), key=lambda r: r["us"])
            return tuple(r["sched"])
        picks = {"schoolbook_best": best(lambda s: s[4] == 0), "schoolbook_radix2_best": best(
            lambda s: s[4] == 0 and s[3] == 1), "karatsuba_best": best(lambda s: s[4] == 1)}
        picks["schoolbook_on_karatsuba_shape"] = picks["karatsuba_best"][:4] + (0,)
        res, ok = {}, True
        for name, sch in picks.items():
            moma.ntt_set_schedule(q, w, n, L, sch)
            us = _time_fwd(moma, torch, stream, dx, dy, q, w, 5, 200)
            ok &= bool((mi.from_planar(dy.cpu().numpy().view(np.uint32)) == want).all())
            res[name] = {"schedule": list(sch), "us": round(us, 3)}
        D = -(-(32 * L - 2) // (29 if L <= 28 else 28))
        h, g = (D + 1) // 2, D // 2
        print(json.dumps({"lambda": lam, "limbs": L, "digits": D, "log2_n": logn,
                          "digit_products_per_multiply": {"schoolbook": 2 * D * D,
                                                          "karatsuba": 2 * h * h + g * g + D * D},
                          **res,
                          "karatsuba_over_schoolbook_best": round(res["karatsuba_best"]["us"] /
                                                                  res["schoolbook_best"]["us"], 3),
                          "karatsuba_over_schoolbook_same_shape": round(
                              res["karatsuba_best"]["us"] / res["schoolbook_on_karatsuba_shape"]["us"], 3),
                          "outputs_vs_oracle": ok}), flush=True)
        moma.ntt_set_schedule(q, w, n, L, None)
        del dx, dy
        moma.shutdown()
    moma.tune_db_clear()


def peaks():
    """The library's issue-rate and bandwidth probes, as rates and as fractions
    of the vendor peaks (39.32 T full-rate lane operations/s, 8 TB/s)."""
    import paper_2501_07535_amd as moma
    r = moma.measure_peaks()
    cm, ca = issue_costs(r)
    out = {"rates_Tops": {k: round(r[k] / 1e12, 3) for k in ("add_u32", "add_co_addc_u32", "mad_u64_u32",
                                                              "mad_addc_u32", "mul_lo_u32", "mul_hi_u32")},
           "of_full_rate": {k: round(r[k] / PEAK_INT_OPS, 4) for k in ("add_u32", "add_co_addc_u32", "mad_u64_u32",
                                                                     "mad_addc_u32", "mul_lo_u32", "mul_hi_u32")},
           "hbm_TBs": {"copy": round(r["hbm_copy"] / 1e12, 3), "triad": round(r["hbm_triad"] / 1e12, 3)},
           "of_hbm_peak": {"copy": round(r["hbm_copy"] / PEAK_HBM, 4), "triad": round(r["hbm_triad"] / PEAK_HBM, 4)},
           "lane_ops_per_word_product_with_carry": round(cm, 4), "lane_ops_per_add_op": round(ca, 4),
           "lane_ops_multiply": {str(L): {k: round(v, 1) for k, v in multiply_forms(L, r).items()}
                                 for L in (2, 4, 8, 12, 16, 24, 32)},
           "lane_ops_per_butterfly": {str(L): round(butterfly_slots(L, r), 1) for L in (2, 4, 8, 12, 16, 24, 32)},
           "compute_units": r["compute_units"]}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the transform path is "
              "single-GPU (the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        sweep(args)
        return
    if args.blas:
        blas(args)
        return
    if args.peaks:
        peaks()
        return
    if args.mulalg:
        mulalg(args)
        return
    import torch

    import paper_2501_07535_amd as moma

    dev = torch.device("cuda:0")
    lam, logn = args.lam, args.logn
    f = mi.find_prime(lam, 0)
    L, n, q = f.limbs, 1 << logn, f.q
    w = f.root(n)
    x = mi.residues(f, n, L, 2, logn)   # same stream as the parity tests
    dx = torch.from_numpy(mi.to_planar(x).view(np.int32)).to(dev)
    dy = torch.empty_like(dx)
    dz = torch.empty_like(dx)
    moma.ntt_prepare(q, w, n, L)
    stream = torch.cuda.current_stream()
    default_sched = moma.ntt_get_schedule(q, w, n, L)
    default_us = None if args.forward_only else _time_fwd(moma, torch, stream, dx, dy, q, w, 3, 20)
    def settle(seconds):
        return _settle_fwd(moma, torch, dx, dy, q, w, seconds)

    tuned = None
    # the autotuner's timings, too, should see the steady clock
    settle_tune_n = 0 if args.schedule or args.no_tune else settle(args.settle)
    if args.schedule:
        moma.ntt_set_schedule(q, w, n, L, tuple(int(v) for v in args.schedule.split(",")))  # 4 or 5 fields
    elif not args.no_tune:
        # the library's autotuner picks the launch shape before the timed region
        tuned = moma.ntt_tune(q, w, n, L, reps=3, warmup=1)
    plan = moma.ntt_describe(q, w, n, L)
    launches = plan["passes"]

    # Clock settle: after the autotuner's timings (short runs with host
    # synchronisations between them) the clock is low again, so untimed
    # transforms run for args.settle seconds before the W warm-up steps and
    # the timed steps see the steady clock.
    settle_n = settle(args.settle)

    for _ in range(args.warmup):
        moma.ntt_fwd(dx, q, w, out=dy)
    torch.cuda.synchronize()

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        moma.ntt_fwd(dx, q, w, out=dy)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps

    # inverse transform timing (not the headline), same protocol
    ms_inv = None
    if not args.forward_only:
        for _ in range(args.warmup):
            moma.ntt_inv(dy, q, w, out=dz)
        ev0.record(stream)
        for _ in range(args.steps):
            moma.ntt_inv(dy, q, w, out=dz)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_inv = ev0.elapsed_time(ev1) / args.steps

    # checks outside the timed region: round trip on the whole vector, and
    # sampled outputs against the oracle's definition
    roundtrip = None if args.forward_only else bool(torch.equal(dz, dx))
    sampled_ok = None
    try:
        import oracle
        ks = np.array([0, 1, n // 3, n - 1], dtype=np.int64)
        got = mi.from_planar(dy[:, torch.from_numpy(ks).to(dev)].cpu().numpy().view(np.uint32))
        sampled_ok = bool((got == oracle.ntt_direct(q, L, w, x, ks)).all())
    except Exception as e:  # the oracle is optional for the measurement itself
        print(f"oracle check skipped: {e}", file=sys.stderr)

    cyc = None if args.forward_only else cyclic_product(moma, torch, stream, dx, dy, dz, q, w, n, args.warmup,
                                                         args.steps)

    B = n // 2 * logn
    gbfly = B / (ms_step * 1e-3) / 1e9
    # the pass kernel's average duration: HIP events over the timed region on
    # the stream the library launches on, divided by the launches it holds
    launch_ms = ms_step / launches
    # issue rates measured on this device after the timed region
    rates = moma.measure_peaks()
    slots = butterfly_slots(L, rates)
    achieved = slots * B / launches / (launch_ms * 1e-3) / 1e12
    peak = PEAK_INT_OPS / 1e12
    counters = committed_counters(lam, logn, moma.ntt_get_schedule(q, w, n, L), plan["stages"])
    valu_issue = None
    if counters and counters.get("sq_insts_valu_per_launch"):
        # wave instructions x 4 cycles each over the SIMD-cycles of one launch
        valu_issue = counters["sq_insts_valu_per_launch"] * 4 / (VALU_SIMDS * CLOCK_HZ * launch_ms * 1e-3)
    cm, ca = issue_costs(rates)
    mf = multiply_forms(L, rates)

    if args.calib_copy_mib:
        src = torch.zeros(args.calib_copy_mib << 18, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    steady = None
    if not args.no_batch:
        steady = steady_state(moma, torch, stream, dx, q, w, n, L, logn, settle=args.settle)

    batch = None
    if not args.no_batch:
        batch = batch_vs_plain(args.batch_jobs, args.batch_reps)

    small = None if args.forward_only else small_call_latency(moma, torch, stream)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(q, L, w, x, n, logn, args.cpu_seconds)

    rec = {
        "metric": "256-bit NTT n=2^20 Gbutterfly/s (bit-exact)" if (lam, logn) == (256, 20)
                  else f"{lam}-bit NTT n=2^{logn} Gbutterfly/s (bit-exact)",
        "value": round(gbfly, 4),
        "unit": "Gbutterfly/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"forward NTT, {lam}-bit class, n=2^{logn}, one transform per step",
                   "lambda": lam, "limbs": L, "q_bits": q.bit_length(), "log2_n": logn,
                   "layout": "limb-planar", "twiddles": "precomputed table"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "Tops/s",
                     "frac": round(achieved / peak, 4),
                     "traffic": counters["traffic_bytes_per_launch"] if counters else None,
                     "kernel": f"ntt_pass_kernel<{L}, radix_log {moma.ntt_get_schedule(q, w, n, L)[3]}>",
                     "launches_per_step": launches,
                     "avg_launch_us": round(launch_ms * 1e3, 3),
                     "avg_launch_us_from": "HIP events over the timed region / launches",
                     "op_model": {"word_products_per_multiply": word_products(L),
                                  "digit_products_per_multiply": 2 * mf["digits"] ** 2,
                                  "lane_ops_multiply_word_form": round(mf["word"], 2),
                                  "lane_ops_multiply_digit_form": round(mf["digit"], 2),
                                  "add_class_ops_per_butterfly": 6 * L,
                                  "lane_ops_per_add_op": round(ca, 4),
                                  "lane_ops_per_butterfly": round(slots, 2)},
                     "measured_rates_Tops": {k: round(rates[k] / 1e12, 3) for k in
                                             ("add_u32", "add_co_addc_u32", "mad_u64_u32", "mad_addc_u32",
                                              "mul_lo_u32", "mul_hi_u32")},
                     "hbm_copy_TBs": round(rates["hbm_copy"] / 1e12, 3),
                     "valu_issue_frac": round(valu_issue, 4) if valu_issue else None,
                     "pass_stages": plan["stages"],
                     "schedule": list(moma.ntt_get_schedule(q, w, n, L))},
        "cpu_baseline": cpu,
        "extras": {"fwd_us": round(ms_step * 1e3, 3), "inv_us": round(ms_inv * 1e3, 3) if ms_inv else None,
                   "clock_settle": {"seconds": args.settle, "untimed_transforms": settle_n,
                                    "before_autotuning": settle_tune_n, "before_each_steady_state_batch": True},
                   "default_schedule": list(default_sched),
                   "default_schedule_fwd_us": round(default_us, 3) if default_us else None,
                   "autotuned": tuned,
                   "ns_per_butterfly_paper_metric": round(2 * ms_step * 1e6 / (n * logn), 6),
                   "hbm_bytes_min_per_step": 2 * n * 4 * L,
                   "roundtrip_exact": roundtrip, "sampled_vs_oracle": sampled_ok,
                   "steady_state": steady,
                   "cyclic_product": cyc,
                   "n2e12_single_call": small,
                   "batched_vs_plain_speedup": batch["speedup"] if batch else None,
                   "batch": batch},
    }
    print(json.dumps(rec), flush=True)


def committed_counters(lam, logn, schedule, stages):
    """The pass kernel's rocprofv3 counters committed under profiles/ (HBM bytes
    per launch from FETCH_SIZE and WRITE_SIZE, VALU wave instructions per
    launch), if they were taken on the current kernel sources with the same
    launches (pass stages, columns per tile, threads and register radix; the
    tile size bound itself does not change the launches); else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"ntt_counters_L{(lam + 31) // 32}_{lam}bit_n2e{logn}.json")
    if not os.path.exists(path):
        return None
    top = json.load(open(path))
    h = hashlib.sha256()
    for f in top["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != top["kernel_sources_sha256"]:
        return None
    # one record per launch shape the autotuner picks at this size
    for rec in top.get("records", []):
        if list(rec["pass_stages"]) == list(stages) and list(rec["schedule"])[1:] == list(schedule)[1:]:
            return rec
    return None


def small_call_latency(moma, torch, stream, reps=100, warmup=10):
    """The 4096-point 256-bit forward and inverse transform as single calls:
    median time per call over `reps` calls after `warmup`, each call bracketed
    by its own events (latency, not throughput), and the round trip."""
    import oracle
    f = mi.find_prime(256, 0)
    L, n, q = f.limbs, 1 << 12, f.q
    w = f.root(n)
    x = mi.residues(f, n, L, 900, 1)
    dx = torch.from_numpy(mi.to_planar(x).view(np.int32)).to(stream.device)
    dy, dz = torch.empty_like(dx), torch.empty_like(dx)
    moma.ntt_prepare(q, w, n, L)
    res = {"schedule": list(moma.ntt_get_schedule(q, w, n, L))}
    for name, fn in (("fwd_us", lambda: moma.ntt_fwd(dx, q, w, out=dy)),
                     ("inv_us", lambda: moma.ntt_inv(dy, q, w, out=dz))):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            t.append(e0.elapsed_time(e1) * 1e3)
        res[name] = round(float(np.median(t)), 3)
    res["roundtrip_exact"] = bool(torch.equal(dz, dx))
    got = mi.from_planar(dy.cpu().numpy().view(np.uint32))
    res["fwd_vs_oracle"] = bool((got == oracle.ntt_radix2(q, L, w, x)).all())
    return res


def cyclic_product(moma, torch, stream, da, db, dc, q, w, n, warmup, reps):
    """Cyclic product a * b mod (x^n - 1) of two resident vectors: the fused call
    (pointwise product inside the inverse transform's first pass) against the
    same steps as four separate calls (fwd, fwd, vmul, inv).  Checked outside
    the timed region: a product with x^s is a rotation by s."""
    ta, tb = torch.empty_like(da), torch.empty_like(da)

    def fused():
        moma.ntt_cyclic_mul(da, db, q, w, out=dc)

    def unfused():
        moma.ntt_fwd(da, q, w, out=ta)
        moma.ntt_fwd(db, q, w, out=tb)
        moma.vmul(ta, tb, q, out=ta)
        moma.ntt_inv(ta, q, w, out=dc)

    for fn in (fused, unfused):
        for _ in range(warmup):
            fn()
    # alternate the two in rounds so that clock and power drift hit both alike
    rounds, per = 5, max(1, reps // 5)
    times = {"fused_us": [], "unfused_us": []}
    for _ in range(rounds):
        for name, fn in (("fused_us", fused), ("unfused_us", unfused)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(per):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            times[name].append(e0.elapsed_time(e1) * 1e3 / per)
    res = {k: round(float(np.median(v)), 3) for k, v in times.items()}
    s = 12345 % n
    shift = torch.zeros_like(da)
    shift[0, s] = 1
    moma.ntt_cyclic_mul(da, shift, q, w, out=dc)
    torch.cuda.synchronize()
    res["shift_is_rotation"] = bool(torch.equal(dc, torch.roll(da, s, dims=1)))
    res["fused_speedup"] = round(res["unfused_us"] / res["fused_us"], 3)
    del ta, tb, shift
    return res


def _settle_fwd(moma, torch, dx, dy, q, w, seconds):
    """Untimed forward transforms for `seconds` (the GPU clock ramps up over
    tens of milliseconds of sustained work and drops in idle gaps)."""
    k = 0
    t0 = time.time()
    while time.time() - t0 < seconds:
        moma.ntt_fwd(dx, q, w, out=dy)
        k += 1
        if k % 32 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return k


def _time_fwd(moma, torch, stream, dx, dy, q, w, warmup, reps):
    for _ in range(warmup):
        moma.ntt_fwd(dx, q, w, out=dy)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        moma.ntt_fwd(dx, q, w, out=dy)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def _settle_batch(torch, b, seconds):
    """Untimed runs of a batch for `seconds`, as _settle_fwd for single calls:
    building the batch leaves the GPU idle and its clock low."""
    k = 0
    t0 = time.time()
    while time.time() - t0 < seconds:
        b.run()
        k += 1
        if k % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return k


def steady_state(moma, torch, stream, dx, q, w, n, L, logn, ks=(1, 2, 4, 8, 16, 32, 64), settle=0.0):
    """The paper's steady-state protocol (Section 5.1): t_single = t_all / k for a
    batch of k transforms of this size, minimised over k; here each batch is one
    graph launch of the batched executor over k independent buffers, timed after
    `settle` seconds of untimed runs of the same batch."""
    outs = [torch.empty_like(dx) for _ in range(max(ks))]
    ins = [dx.clone() for _ in range(max(ks))]
    res = {}
    for k in ks:
        b = moma.Batch([(ins[i], outs[i], q, w, False) for i in range(k)])
        b.run()
        torch.cuda.synchronize()
        _settle_batch(torch, b, settle)
        reps = max(3, 32 // k)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.run()
        e1.record(stream)
        torch.cuda.synchronize()
        res[k] = e0.elapsed_time(e1) * 1e3 / reps / k
        b.close()
    same = all(torch.equal(outs[i], outs[0]) for i in range(max(ks)))
    kbest = min(res, key=res.get)
    B = n // 2 * logn
    return {"us_per_transform_by_k": {str(k): round(v, 3) for k, v in res.items()}, "best_k": kbest,
            "us_per_transform": round(res[kbest], 3), "gbutterfly_s": round(B / (res[kbest] * 1e-6) / 1e9, 3),
            "outputs_identical": same}


def batch_vs_plain(njobs: int, reps: int):
    """The batched workload: njobs transforms, log2 n uniform in 10..16, widths
    {64,128,256,384} bits, each with its own prime.  Plain = one moma_ntt_fwd C
    call per job on one stream (arguments prebuilt, so the loop is the library's
    own per-call cost); batched = one moma_batch_run (one graph launch).  Both
    timed with events on the stream, plans built beforehand."""
    import ctypes

    import torch

    import paper_2501_07535_amd as moma
    jobs = mi.batch_jobs(njobs)
    xs = mi.batch_inputs(jobs)
    dev = torch.device("cuda:0")
    dx = [torch.from_numpy(mi.to_planar(x).view(np.int32)).to(dev) for x in xs]
    del xs
    outs_plain = [torch.empty_like(x) for x in dx]
    outs_batch = [torch.empty_like(x) for x in dx]
    lib = moma.library()
    args = []
    for j, x, o in zip(jobs, dx, outs_plain):
        L = j.limbs
        qw, ww = moma._words(j.field.q, L), moma._words(j.omega, L)
        moma.ntt_prepare(j.field.q, j.omega, j.n, L)
        args.append((qw, ww, j.n, L, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(o.data_ptr())))
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    fwd = lib.moma_ntt_fwd

    def plain():
        for a in args:
            rc = fwd(a[0], a[1], a[2], a[3], a[4], a[5], sp)
            if rc:
                raise moma.MomaError(rc)

    t0 = time.perf_counter()
    b = moma.Batch([(x, o, j.field.q, j.omega, False) for j, x, o in zip(jobs, dx, outs_batch)])
    t_create = time.perf_counter() - t0
    plain()
    b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plain()
    e1.record(stream)
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) / reps
    e0.record(stream)
    for _ in range(reps):
        b.run()
    e1.record(stream)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / reps
    same = all(torch.equal(p, q) for p, q in zip(outs_plain, outs_batch))
    bfly = sum(j.n // 2 * j.logn for j in jobs)
    info = b.info()
    b.close()
    return {"jobs": njobs, "plain_ms": round(t_plain, 4), "batched_ms": round(t_batch, 4),
            "speedup": round(t_plain / t_batch, 3), "batched_gbutterfly_s": round(bfly / (t_batch * 1e-3) / 1e9, 3),
            "graph_launches": info["launches"], "tiles": info["items"], "create_s": round(t_create, 2),
            "outputs_identical": same}


def cpu_baseline(q, L, w, x, n, logn, seconds):
    """The oracle's whole-vector transform, repeated for about `seconds` on the host cores."""
    try:
        import oracle
    except Exception as e:
        print(f"cpu baseline skipped: {e}", file=sys.stderr)
        return None
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.ntt_radix2(q, L, w, x)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    per = el / reps
    return {"value": round(n // 2 * logn / per / 1e9, 6), "unit": "Gbutterfly/s", "cores": oracle.threads(),
            "kind": "oracle", **host_cpu(),
            "sample": f"the full n=2^{logn} forward transform (oracle radix-2, division-based modmul), "
                      f"{reps} repetitions, {el:.1f} s"}


if __name__ == "__main__":
    main()
