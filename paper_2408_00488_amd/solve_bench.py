"""Timing of single persistent solves of the named workloads, one JSON line
per case: the problem autotuner's schedule (or a fixed one), then `reps`
solves timed with HIP events on the solve's stream.  Used for the solver's
kernel traces and HBM counters on one system at a time.

Algorithmic bytes per grid point and MINRES iteration: stencil 40 + Lanczos
recurrence and w / x updates 160 + 4 s bytes per sine-transform pass (s = 8
FP64, 4 FP32 preconditioner): 3 passes in 2-D and in 3-D with the plane phase
(the two leading axes' plane transformed in one pass: 296 FP64, 248 FP32), 5
in 3-D otherwise (360 FP64, 280 FP32).

  python -m paper_2408_00488_amd.solve_bench [--cases c3,c3_fp32] [--reps 5] [--dst fft]
                                             [--tile-points P --lds L --threads T]
"""
from __future__ import annotations

import argparse
import json



def bytes_per_point_iter(d: int, fp32: bool, plane: bool) -> float:
    return 200.0 + (3 if d == 2 or plane else 5) * 4.0 * (4 if fp32 else 8)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="c3,c3_fp32")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--tile-points", type=int, default=-1,
                    help="fixed schedule (with --lds, --threads) instead of the autotuner")
    ap.add_argument("--lds", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--dst", default="auto", help="sine-transform engine: auto, fft, gemm, gemm16")
    args = ap.parse_args()
    import torch
    import paper_2408_00488_amd as C
    from paper_2408_00488_amd import workloads as WL
    C.load_library()
    dev = torch.device("cuda:0")
    for case in args.cases.split(","):
        name, _, prec = case.partition("_")
        fp32 = prec == "fp32"
        s = WL.workload(name).systems[0]
        a = torch.from_numpy(s.a).to(dev)
        f = torch.from_numpy(s.f).to(dev)
        z = torch.empty_like(f)
        p = C.Problem(a, s.lam.real, s.lam.imag, pinv_fp32=fp32, dst=args.dst)
        if args.tile_points >= 0:
            p.set_schedule(args.tile_points, args.lds, args.threads)
        else:
            p.tune(f, z)
        _, info = C.minres_solve(p, f, z)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.reps):
            C.minres_solve(p, f, z, want_info=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.reps
        bpp = bytes_per_point_iter(s.a.ndim, fp32, p.schedule["block_threads"] == 1024)
        alg = info["iters"] * s.a.size * bpp
        print(json.dumps({"case": case, "points": int(s.a.size), "iters": info["iters"],
                          "relres_true": info["relres_true"], "ms_per_solve": round(ms, 4),
                          "bytes_per_point_iter": bpp, "alg_bytes_per_solve": alg,
                          "alg_GBps": round(alg / ms / 1e6, 1),
                          "frac_of_8TBps": round(alg / ms / 1e6 / 8000.0, 4),
                          "schedule": p.schedule, "engines": list(p.dst_engines)}),
              flush=True)
        p.close()


if __name__ == "__main__":
    main()
