"""Timing of the sine-transform engines inside the batched solver.

Solves `count` copies of a 2-D system on an n x n grid (coefficient and
shifts as in the batched-shift workload) in one batched launch with every
axis on the chosen engine, and prints one JSON line: time per batched
solve, solves/s, iterations, and the matrix-core flops the GEMM engine
issues per solve (8 hp^2 per line transform, hp = ceil(n/2) rounded up to
16: re and im columns times the even and odd halves of the first ceil(n/2)
rows; four line transforms of n lines per iteration in 2-D; the FP16
split-product engine, gemm16, issues three products for each, the FP64 row
pass of the Lanczos vectors keeping one FP64 product).  Used to pick the engine
per axis by measurement and to read MFMA utilisation under rocprofv3.

  python -m paper_2408_00488_amd.dst_bench --engine gemm --n 127 --count 64 [--fp32]
  python -m paper_2408_00488_amd.dst_bench --engine gemm16 --n 127 --count 64 --fp32
"""
from __future__ import annotations

import argparse
import json
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--engine", choices=["fft", "gemm", "gemm16"], default="gemm")
    ap.add_argument("--n", type=int, default=127)
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--fp32", action="store_true")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import torch
    import paper_2408_00488_amd as C
    from paper_2408_00488_amd import workloads as WL
    C.load_library()
    dev = torch.device("cuda:0")
    n, cnt = args.n, args.count
    a = torch.from_numpy(WL.coef_c1(n)).to(dev)
    lams = WL.batched_shifts(cnt, 1e-2, 1.0 / 64)
    g = WL.rng(7)
    probs, F = [], []
    for j in range(cnt):
        probs.append(C.Problem(a, lams[j].real, lams[j].imag, pinv_fp32=args.fp32,
                               dst=args.engine))
        F.append(torch.from_numpy(WL.complex_normal(g, (n, n))).to(dev))
    Z = [torch.empty_like(f) for f in F]
    b = C.Batch(probs, timeout_ms=60000)
    _, infos = b.solve(F, Z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.reps):
        b.solve(F, Z, want_info=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.reps * 1e3
    iters = sum(i["iters"] for i in infos)
    # per line transform: re and im columns, even and odd halves of the first
    # ceil(n/2) rows (padded to hp), 2 flops per product; 4 passes of n lines
    hp = ((n + 1) // 2 + 15) // 16 * 16
    per_pass = n * 8 * hp * hp * iters
    if args.engine == "gemm":
        flops = 4 * per_pass
    elif args.engine == "gemm16":
        # three FP16 products in the three preconditioner passes, one FP64
        # product in the row pass of the Lanczos vectors
        flops = 3 * 3 * per_pass + per_pass
    else:
        flops = 0
    print(json.dumps({"engine": args.engine, "n": n, "count": cnt, "fp32": args.fp32,
                      "engines": list(probs[0].dst_engines), "ms_per_solve": ms,
                      "solves_per_s": cnt / ms * 1e3, "iters": iters,
                      "max_relres": max(i["relres_true"] for i in infos),
                      "gemm_flops_per_solve": flops,
                      "gemm_tflops": flops / ms / 1e9 if flops else 0.0}), flush=True)
    b.close()
    for p in probs:
        p.close()


if __name__ == "__main__":
    main()
