"""Build the tuning database, train the cost model on it, and measure its regret.

  python -m paper_2501_07535_amd.tuning collect --db DB.csv --widths 64:1024:32 --logn 10:26 [--max-seconds S]
      exhaustive autotuning of every (bit-width class, size) shape, appended to DB.csv
      (shapes already in DB.csv are skipped, so an interrupted collection resumes)
  python -m paper_2501_07535_amd.tuning evaluate --db DB.csv [DB2.csv ...] --out report.json --model cm.txt
      hold out shapes, train the model on the rest (on the GPU), and report the
      regret of timing only the model's top-k shapes against exhaustive search
  python -m paper_2501_07535_amd.tuning train --db DB.csv [...] --model cm.txt
      train the cost model on every shape (the model a package ships: new plans
      without timings start from its top-ranked schedule)
  python -m paper_2501_07535_amd.tuning picks --db DB.csv [...] --model cm.txt --out picks.json
      the top-1 regret of a saved model on every shape of the database (for the
      packaged model: the cost of a new plan's first pick on shapes it was trained on)
  python -m paper_2501_07535_amd.tuning widths --db DB.csv [...] --out widths.json
      the autotuned transform time against the bit-width class at fixed sizes,
      and the slowdown per doubling of the width (Section 5.4); no GPU needed

Regret of a shape = t(fastest of the model's top-k) / t(fastest of all) - 1, with
both times taken from the same exhaustive sweep.  The comparison baselines spend
the same k timings on k schedules drawn at random (expected regret over all
k-subsets) or on the library's default schedule alone.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from itertools import combinations

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _rng_range(s: str):
    a, b, *c = [int(v) for v in s.split(":")]
    return list(range(a, b + 1, c[0] if c else 1))


def collect(db: str, widths, logns, reps: int, warmup: int, max_seconds: float = 0.0):
    import moma_inputs as mi
    import paper_2501_07535_amd as moma
    if os.path.exists(db):
        moma.tune_db_load(db)
    done = {(r["limbs"], r["log2_n"]) for r in moma.tune_db_rows()}
    t0 = time.time()
    for lam in widths:
        f = mi.find_prime(lam, 4)
        L = f.limbs
        for logn in logns:
            if (L, logn) in done:
                continue
            if max_seconds and time.time() - t0 > max_seconds:
                print(f"stopping after {time.time() - t0:.0f}s (--max-seconds); rerun to continue", flush=True)
                return len(moma.tune_db_rows())
            n = 1 << logn
            r = moma.ntt_tune(f.q, f.root(n), n, L, reps=reps, warmup=warmup)
            print(f"[{time.time() - t0:7.1f}s] lam={lam} L={L} logn={logn} timed={r['timed']} "
                  f"best={r['best']} {r['best_us']:.1f}us", flush=True)
            moma.tune_db_save(db)
        moma.shutdown()   # drop this width's plans and tables
    return len(moma.tune_db_rows())


def load_rows(paths):
    rows = []
    for p in paths:
        with open(p) as fh:
            next(fh)
            for line in fh:
                # device,limbs,log2_n,tile_log,col_log,threads,radix_log,us,reps[,mul_variant]
                v = line.strip().split(",")
                mv = int(v[9]) if len(v) > 9 else 0
                rows.append((int(v[1]), int(v[2]), (int(v[3]), int(v[4]), int(v[5]), int(v[6]), mv), float(v[7])))
    # latest measurement of each (shape, schedule)
    last = {}
    for L, logn, s, us in rows:
        last[(L, logn, s)] = us
    return [(k[0], k[1], k[2], v) for k, v in last.items()]


def evaluate(paths, out, model_path, ks=(1, 3, 5, 10), holdout=0.2, seed=7, epochs=300, batch=256, lr=3e-3):
    import moma_inputs as mi
    import paper_2501_07535_amd as moma
    rows = load_rows(paths)
    shapes = sorted({(L, n) for L, n, _, _ in rows})
    maxL = max(L for L, _ in shapes)
    maxn = max(n for _, n in shapes)
    # held out: a seeded 20% of shapes, plus the largest size and the widest class (extrapolation)
    u = mi.uniform01(len(shapes), 8, seed)
    extra = {s for s in shapes if s[0] == maxL or s[1] == maxn}
    held = {s for s, v in zip(shapes, u) if v < holdout} | extra
    train = [r for r in rows if (r[0], r[1]) not in held]
    feats = np.array([moma.costmodel_features(L, n, s) for L, n, s, _ in train], np.float32)
    y = np.log(np.array([us for *_, us in train], np.float32))
    t0 = time.time()
    mse = moma.costmodel_train(feats, y, epochs=epochs, batch=batch, lr=lr, seed=seed)
    train_s = time.time() - t0
    if model_path:
        moma.costmodel_save(model_path)
    by_shape = {}
    for L, n, s, us in rows:
        by_shape.setdefault((L, n), []).append((s, us))
    report = {"rows": len(rows), "shapes": len(shapes), "train_rows": len(train), "heldout_shapes": len(held),
              "extrapolation_shapes": len(extra), "train_mse_log_us": mse, "train_seconds": round(train_s, 2),
              "k": {}}
    for k in ks:
        reg_model, reg_rand, reg_default, saved = [], [], [], 0
        for shp in sorted(held):
            cands = by_shape[shp]
            times = np.array([us for _, us in cands])
            best = times.min()
            f = np.array([moma.costmodel_features(shp[0], shp[1], s) for s, _ in cands], np.float32)
            pred = moma.costmodel_predict(f)
            order = np.argsort(pred, kind="stable")
            kk = min(k, len(cands))
            reg_model.append(times[order[:kk]].min() / best - 1)
            # expected best of a uniformly random k-subset: E[min] from the order statistics
            srt = np.sort(times)
            m = len(srt)
            probs = [math.comb(m - 1 - i, kk - 1) / math.comb(m, kk) for i in range(m)]
            reg_rand.append(float(np.dot(probs, srt)) / best - 1)
            d = default_schedule_time(moma, shp, cands)
            if d is not None:
                reg_default.append(d / best - 1)
            saved += len(cands) - kk
        gm = lambda v: float(np.exp(np.mean(np.log1p(np.array(v)))) - 1) if v else None
        report["k"][str(k)] = {"geomean_regret_model": gm(reg_model), "max_regret_model": float(max(reg_model)),
                               "geomean_regret_random_k": gm(reg_rand), "geomean_regret_default": gm(reg_default),
                               "timings_saved": saved,
                               "within_5pct_fraction": float(np.mean(np.array(reg_model) <= 0.05))}
    with open(out, "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps(report, indent=1), flush=True)
    return report


def train_all(paths, model_path, seed=7, epochs=300, batch=256, lr=3e-3):
    import paper_2501_07535_amd as moma
    rows = load_rows(paths)
    feats = np.array([moma.costmodel_features(L, n, s) for L, n, s, _ in rows], np.float32)
    y = np.log(np.array([us for *_, us in rows], np.float32))
    t0 = time.time()
    mse = moma.costmodel_train(feats, y, epochs=epochs, batch=batch, lr=lr, seed=seed)
    moma.costmodel_save(model_path)
    print(json.dumps({"rows": len(rows), "train_mse_log_us": mse, "train_seconds": round(time.time() - t0, 2),
                      "model": model_path}), flush=True)


def picks(paths, model_path, out):
    import paper_2501_07535_amd as moma
    moma.costmodel_load(model_path)
    by_shape = {}
    for L, n, s, us in load_rows(paths):
        by_shape.setdefault((L, n), []).append((s, us))
    regret, picked = [], {}
    for shp in sorted(by_shape):
        cands = by_shape[shp]
        times = np.array([us for _, us in cands])
        f = np.array([moma.costmodel_features(shp[0], shp[1], s) for s, _ in cands], np.float32)
        i = int(np.argmin(moma.costmodel_predict(f)))
        regret.append(float(times[i] / times.min() - 1))
        picked[f"{shp[0]},{shp[1]}"] = {"pick": list(cands[i][0]), "regret": round(regret[-1], 4)}
    r = np.array(regret)
    report = {"shapes": len(r), "geomean_regret": float(np.exp(np.mean(np.log1p(r))) - 1),
              "max_regret": float(r.max()), "within_5pct_fraction": float(np.mean(r <= 0.05)),
              "radix16_picks": sum(1 for v in picked.values() if v["pick"][3] == 4), "by_shape": picked}
    with open(out, "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps({k: v for k, v in report.items() if k != "by_shape"}, indent=1), flush=True)
    return report


def widths(paths, out, logns=(12, 16)):
    """Autotuned (fastest measured) time per bit-width class at fixed n, and the
    slowdown factor of each width doubling 64 -> 128 -> ... -> 1024."""
    rows = load_rows(paths)
    best = {}
    for L, n, _, us in rows:
        best[(L, n)] = min(us, best.get((L, n), float("inf")))
    report = {"note": "class width = 32 x compute limbs (modulus of width - 4 bits)", "sizes": {}}
    for logn in logns:
        curve = {32 * L: round(us, 3) for (L, n), us in sorted(best.items()) if n == logn}
        doublings = {}
        w = 64
        while 2 * w <= 1024:
            if w in curve and 2 * w in curve:
                doublings[f"{w}->{2 * w}"] = round(curve[2 * w] / curve[w], 3)
            w *= 2
        report["sizes"][str(logn)] = {"us_by_width": curve, "slowdown_per_doubling": doublings}
    with open(out, "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps(report, indent=1), flush=True)
    return report


def default_schedule_time(moma, shp, cands):
    """Time of the schedule a fresh plan would pick by default for this shape, if it was measured."""
    from paper_2501_07535_amd import _default_schedule_for
    s = _default_schedule_for(shp[0], shp[1])
    for c, us in cands:
        if tuple(c) == tuple(s):
            return us
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--db", required=True)
    c.add_argument("--widths", default="64:1024:32")
    c.add_argument("--logn", default="10:26")
    c.add_argument("--reps", type=int, default=3)
    c.add_argument("--warmup", type=int, default=1)
    c.add_argument("--max-seconds", type=float, default=0.0,
                   help="stop before the next shape once this much time has passed (the database keeps what is done)")
    e = sub.add_parser("evaluate")
    e.add_argument("--db", nargs="+", required=True)
    e.add_argument("--out", required=True)
    e.add_argument("--model", default=None)
    e.add_argument("--epochs", type=int, default=300)
    t = sub.add_parser("train")
    t.add_argument("--db", nargs="+", required=True)
    t.add_argument("--model", required=True)
    t.add_argument("--epochs", type=int, default=300)
    p = sub.add_parser("picks")
    p.add_argument("--db", nargs="+", required=True)
    p.add_argument("--model", required=True)
    p.add_argument("--out", required=True)
    w = sub.add_parser("widths")
    w.add_argument("--db", nargs="+", required=True)
    w.add_argument("--out", required=True)
    w.add_argument("--logn", default="12,16")
    a = ap.parse_args()
    if a.cmd == "train":
        train_all(a.db, a.model, epochs=a.epochs)
    elif a.cmd == "picks":
        picks(a.db, a.model, a.out)
    elif a.cmd == "widths":
        widths(a.db, a.out, tuple(int(v) for v in a.logn.split(",")))
    elif a.cmd == "collect":
        n = collect(a.db, _rng_range(a.widths), _rng_range(a.logn), a.reps, a.warmup, a.max_seconds)
        print(f"database rows: {n}", flush=True)
    else:
        evaluate(a.db, a.out, a.model, epochs=a.epochs)


if __name__ == "__main__":
    main()
