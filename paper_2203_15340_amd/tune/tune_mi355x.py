#!/usr/bin/env python3
"""Rebuild the committed launch table (gram_mi355x.json) on one MI355X.

Keeps the table's FP64 Gram entries (chosen by timing the paper form's whole
two-part launch, which the single-block sweep does not see) and sweeps, on the
benchmark's own inputs, the mixed-precision Gram A1^T A1 (the mixed
correction form's only product: split-K tiles and workgroups, and the
persistent kind on an FP32 copy of A1), the residual A^T J (b - A x) of the
20000 x 1000 problem and the batched solver on the 4096-problem batch (FP64
paper form and mixed correction form, stopped at rel.err 1e-6 as in the
benchmark).  Writes the merged table to the path given (default: this
directory's gram_mi355x.json) and prints every entry.

    python paper_2203_15340_amd/tune/tune_mi355x.py [--out PATH]
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def main():
    import numpy as np
    import torch

    import paper_2203_15340_amd as ils
    import workloads as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "gram_mi355x.json"))
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    src = os.path.join(HERE, "gram_mi355x.json")
    ils.tune_clear()
    ils.tune_load(src)
    with open(src) as f:
        gram_entries = [e for e in json.load(f)["entries"] if e["kernel"] == "gram" and e["precision"] == 0]

    P = W.large(ratio=0.5, seed=1)
    A = torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda().t()
    b = torch.from_numpy(P.b).cuda()
    x = torch.from_numpy(np.random.default_rng(0).standard_normal(P.n)).cuda()
    print("mixed Gram:", ils.tune_gram(A, 0, P.p, precision=ils.PREC_MIXED, reps=10), flush=True)
    print("residual:", ils.tune_residual(A, b, P.p, x, reps=10), flush=True)
    del A, b, x

    B = W.batched(4096, seed=3, threads=len(os.sched_getaffinity(0)))
    dv = [(torch.from_numpy(np.ascontiguousarray(Q.A.T)).cuda().t(), torch.from_numpy(Q.b).cuda(), Q.p) for Q in B]
    xr = [torch.from_numpy(Q.x_star).cuda() for Q in B]
    plan = ils.BatchPlan(dv, x_refs=xr)
    kw = dict(stop_rule=ils.STOP_XREF, tol=1e-6)
    for form, prec in ((ils.FORM_PAPER, ils.PREC_FP64), (ils.FORM_CORRECTION, ils.PREC_MIXED)):
        print("batched:", ils.tune_batched(plan, reps=args.reps, form=form, precision=prec, **kw), flush=True)

    ils.tune_save(args.out)
    with open(args.out) as f:
        saved = json.load(f)["entries"]
    # the FP64 Gram entries are the loaded ones, unchanged
    assert sorted(json.dumps(e, sort_keys=True) for e in saved if e["kernel"] == "gram" and e["precision"] == 0) == \
        sorted(json.dumps(dict(e, kind=e.get("kind", 0)), sort_keys=True) for e in gram_entries)
    for e in saved:
        print(json.dumps(e))


if __name__ == "__main__":
    main()
