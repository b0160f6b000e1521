"""Autotuner of the ragged-batch size buckets: leaf size and rank per bucket, per precision.

For each precision form (FP64; the batched FP32 form, whose table the BF16 and FP16 hi+lo
forms share) it takes the transforms of the configuration-4 batch (2048 lengths
log-uniform in [128, 262144], directions 50/50, f_j = z_j/(j+1)) whose lengths fall in
each size bucket, plans them as one ragged batch per candidate (leaf size, rank), times
cold executes, and checks the outputs against an accurate reference computed on the same
GPU (the FP64 path at rank 24).  A candidate counts only if its error E_inf (Eq. (Einf))
stays within the form's bound; the fastest one wins the bucket.  The winners are written
as the library's table (csrc/l2c_tuning_table.h, used when a ragged batch is planned with
tuning = NULL) and a summary of every candidate's time and error (markdown).

    python -m paper_2411_00033_amd.autotune --out-dir <dir>

The table takes effect after the library is rebuilt.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

BUCKETS = [512, 2048, 8192, 32768, 131072, 1 << 62]
CANDIDATES = {
    # rank 16 with leaf <= 64 runs batches of 16 or more in the FP64 tile form
    "fp64": [(leaf, rank) for leaf in (32, 48, 64, 96, 128) for rank in (18, 20)] + [(32, 16), (48, 16), (64, 16)],
    "batched": [(leaf, rank) for leaf in (32, 48, 64) for rank in (12, 16)],
}
BOUND = {"fp64": 1e-13, "batched": 2.5e-6}   # the forms' parity bounds


def _timed(torch, fn, reps, flush, sink):
    stream = torch.cuda.current_stream()
    st = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    en = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    fn()
    torch.cuda.synchronize()
    for i in range(reps):
        torch.sum(flush, dim=0, out=sink)
        st[i].record(stream)
        fn()
        en[i].record(stream)
    torch.cuda.synchronize()
    return float(np.median([st[i].elapsed_time(en[i]) for i in range(reps)]))


def header(tables, note):
    rows = {}
    for form, tab in tables.items():
        rows[form] = ",\n                                      ".join(
            "{%s, %d, %d}" % ("INT64_MAX" if n >= (1 << 62) else str(n), leaf, rank) for n, leaf, rank in tab)
    return """// l2c_tuning_table.h -- leaf size and rank per size bucket of a ragged batch
// (leg2cheb_batch_plan with tuning = NULL), per precision form.
//
// Written by paper_2411_00033_amd/autotune.py from timings of the ragged batch on an
// MI355X; regenerate it with that script.  Each row covers the lengths n with
// n_max(previous row) < n <= n_max; the last row covers every larger n.  Every row met its
// form's error bound against the FP64 path at rank 24 on the bucket's transforms (FP64:
// E_inf <= 1e-13); the batched forms keep rank <= 16 and leaf <= 64.
// %s
#pragma once
#include <stdint.h>

namespace l2c {

struct TuneRow {
    int64_t n_max;
    int32_t leaf_size, rank;
};

static const TuneRow kTuneFP64[] = {%s};
static const TuneRow kTuneBatched[] = {%s};

inline int builtin_tuning(int precision, const TuneRow **rows)
{
    if (precision == 0) {
        *rows = kTuneFP64;
        return (int)(sizeof(kTuneFP64) / sizeof(kTuneFP64[0]));
    }
    *rows = kTuneBatched;
    return (int)(sizeof(kTuneBatched) / sizeof(kTuneBatched[0]));
}

}  // namespace l2c
""" % (note, rows["fp64"], rows["batched"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out-dir", required=True)
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args()
    import torch
    import paper_2411_00033_amd as l2c
    from paper_2411_00033_amd import inputs
    os.makedirs(args.out_dir, exist_ok=True)
    sizes, dirs = inputs.ragged_sizes(2048, inputs.SEED_BASE + 4)
    rng = np.random.default_rng(inputs.SEED_BASE + 5)
    flush = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    sink = torch.empty((), dtype=torch.float64, device="cuda")
    lines = ["# Autotuner of the ragged-batch size buckets (leaf size, rank)", "",
             "command: python -m paper_2411_00033_amd.autotune --out-dir <out>", "",
             "Per form and bucket: every candidate's median cold execute time of the bucket's",
             "transforms of the 2048-transform batch, as one ragged batch, and its E_inf against the",
             "FP64 path at rank 24 (leaf 64) on the same inputs; '*' marks the winner (fastest",
             "within the bound).", ""]
    tables, record = {}, {}
    lo = 0
    bucket_items = []
    for hi in BUCKETS:
        idx = np.flatnonzero((sizes > lo) & (sizes <= hi))
        bucket_items.append((lo, hi, idx))
        lo = hi
    for form, prec in (("fp64", l2c.L2C_FP64), ("batched", l2c.L2C_FP32)):
        tab = []
        lines += ["## %s" % ("FP64" if form == "fp64" else "batched forms (timed in FP32)"), "",
                  "| bucket n | transforms | leaf | rank | ms | E_inf |", "|---|---|---|---|---|---|"]
        for lo, hi, idx in bucket_items:
            if idx.size == 0:
                continue
            ns, ds = sizes[idx], dirs[idx]
            offs = np.concatenate([[0], np.cumsum(ns)])
            flat = rng.standard_normal(int(offs[-1]))
            for i, n in enumerate(ns):
                flat[offs[i]:offs[i + 1]] /= np.arange(1, n + 1, dtype=np.float64)
            x = torch.from_numpy(flat).cuda()
            y = torch.empty_like(x)
            ref = torch.empty_like(x)
            ip = [x.data_ptr() + 8 * int(o) for o in offs[:-1]]
            op = [y.data_ptr() + 8 * int(o) for o in offs[:-1]]
            rp = [ref.data_ptr() + 8 * int(o) for o in offs[:-1]]
            with l2c.BatchPlan(ns.tolist(), ds.tolist(), precision=l2c.L2C_FP64, tuning=[(1 << 62, 64, 24)]) as bp:
                bp.execute_ptrs(ip, rp)
                torch.cuda.synchronize()
            rh = ref.cpu().numpy()
            best = None
            rows = []
            for leaf, rank in CANDIDATES[form]:
                with l2c.BatchPlan(ns.tolist(), ds.tolist(), precision=prec, tuning=[(1 << 62, leaf, rank)]) as bp:
                    ms = _timed(torch, lambda: bp.execute_ptrs(ip, op), args.reps, flush, sink)
                yh = y.cpu().numpy()
                err = max(float(np.max(np.abs(yh[offs[i]:offs[i + 1]] - rh[offs[i]:offs[i + 1]]))
                                / max(np.max(np.abs(rh[offs[i]:offs[i + 1]])), 1e-300)) for i in range(len(ns)))
                rows.append((leaf, rank, ms, err))
                if err <= BOUND[form] and (best is None or ms < best[2]):
                    best = (leaf, rank, ms, err)
                print("%s bucket (%d, %d] leaf %d rank %d: %.4f ms E_inf %.2e" % (form, lo, hi, leaf, rank, ms, err),
                      flush=True)
            if best is None:
                best = (64, 18 if form == "fp64" else 16, 0.0, 0.0)
            tab.append((hi, best[0], best[1]))
            for leaf, rank, ms, err in rows:
                mark = "*" if (leaf, rank) == best[:2] else ""
                lines.append("| (%d, %s] | %d | %d%s | %d | %.4f | %.2e |" % (
                    lo, "inf" if hi >= (1 << 62) else str(hi), idx.size, leaf, mark, rank, ms, err))
            record.setdefault(form, []).append({"bucket": [lo, hi], "rows": rows, "best": best})
        # merge neighbouring buckets with the same winner
        merged = []
        for row in tab:
            if merged and merged[-1][1:] == row[1:]:
                merged[-1] = row
            else:
                merged.append(row)
        tables[form] = merged
        lines += ["", "table: %s" % json.dumps(merged), ""]
    stamp = "Made %s UTC." % time.strftime("%Y-%m-%d %H:%M", time.gmtime())
    open(os.path.join(args.out_dir, "l2c_tuning_table.h"), "w").write(header(tables, stamp))
    open(os.path.join(args.out_dir, "autotune_ragged_2048.md"), "w").write("\n".join(lines) + "\n")
    json.dump(record, open(os.path.join(args.out_dir, "autotune.json"), "w"))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
