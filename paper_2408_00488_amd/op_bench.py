"""Bandwidth of the stand-alone operators: the stencil y = A x (apply_A) and
the preconditioner y = P^{-1} x (apply_Pinv, its sine-transform passes and
the per-mode scaling), one JSON line per case.

Model bytes per grid point (complex FP64 vectors of 16 B):
  apply_A     40  (x 16 in, nodal coefficient 8, y 16 out)
  apply_Pinv  per transform pass, read + write of the pass's vector:
              FP64 32; FP32 16, plus 8 on the first and the last pass for
              the FP64 input and output.  2-D 3 passes, 3-D 5 passes:
              2-D FP64 96, 2-D FP32 64, 3-D FP64 160, 3-D FP32 96.
  step transform (op T, the all-at-once layer's paradiag_transform over
              --steps steps, forward and inverse in turn): 32 per point and
              step (read and write of a complex FP64 value); 2-D cases only
              (the layer holds one problem per step).
Times are CUDA-event averages over `reps` back-to-back launches (launch
gaps included); under rocprofv3 --kernel-trace the per-kernel durations of
the same run give the kernels alone.  3-D n = 255 has vectors of 265 MB,
larger than the 256 MB Infinity Cache, so its rate is an HBM rate.

  python -m paper_2408_00488_amd.op_bench [--cases 3d255,3d127,2d1023] [--reps 20] [--lds 65536]
                                          [--ops A,P64,P32,T] [--steps 64]
"""
from __future__ import annotations

import argparse
import json

CASES = {
    "3d255": (255, 255, 255),
    "3d127": (127, 127, 127),
    "2d1023": (1023, 1023),
    "2d511": (511, 511),
}


def pinv_bytes(d: int, fp32: bool) -> float:
    passes = 3 if d == 2 else 5
    return passes * 16.0 + 16.0 if fp32 else passes * 32.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="3d255,3d127,2d1023")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--ops", default="A,P64,P32")
    ap.add_argument("--lds", type=int, default=0,
                    help="LDS line budget of the problems' schedule (0 = default, 65536)")
    ap.add_argument("--steps", type=int, default=64, help="steps of the step transform (op T)")
    args = ap.parse_args()
    import torch
    import paper_2408_00488_amd as C
    from paper_2408_00488_amd import workloads as WL
    C.load_library()
    dev = torch.device("cuda:0")
    ops = args.ops.split(",")
    for name in args.cases.split(","):
        shape = CASES[name]
        M = 1
        for n in shape:
            M *= n
        g = WL.rng(11)
        a = torch.from_numpy(g.uniform(1.0, 3.0, shape)).to(dev)
        x = torch.from_numpy(WL.complex_normal(g, shape)).to(dev)
        y = torch.empty_like(x)
        for op in ops:
            if op == "T":
                if len(shape) != 2:
                    continue
                L = args.steps
                pd = C.ParaDiag(a, L, 1.0 / L, 1e-2, dst="fft")
                xs = torch.from_numpy(WL.complex_normal(g, (L,) + shape)).to(dev)
                ys = torch.empty_like(xs)
                for _ in range(3):
                    pd.transform(xs, ys)
                    pd.transform(ys, xs, inverse=True)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(args.reps):
                    pd.transform(xs, ys)
                    pd.transform(ys, xs, inverse=True)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / (2 * args.reps)
                bpp = 32.0 * L
                print(json.dumps({"case": name, "op": "T", "steps": L, "points": M,
                                  "ms": round(ms, 4), "model_bytes_per_point": bpp,
                                  "model_GBps": round(bpp * M / ms / 1e6, 1),
                                  "frac_of_8TBps": round(bpp * M / ms / 1e6 / 8000.0, 3)}),
                      flush=True)
                pd.close()
                continue
            fp32 = op == "P32"
            p = C.Problem(a, 10.0, 100.0, pinv_fp32=fp32, dst="fft")
            if args.lds:
                p.set_schedule(0, args.lds)
            fn = (lambda: C.apply_A(p, x, y)) if op == "A" else (lambda: C.apply_Pinv(p, x, y))
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.reps
            bpp = 40.0 if op == "A" else pinv_bytes(len(shape), fp32)
            print(json.dumps({"case": name, "op": op, "lds": p.schedule["lds_bytes"],
                              "points": M, "ms": round(ms, 4),
                              "model_bytes_per_point": bpp,
                              "model_GBps": round(bpp * M / ms / 1e6, 1),
                              "frac_of_8TBps": round(bpp * M / ms / 1e6 / 8000.0, 3)}),
                  flush=True)
            p.close()


if __name__ == "__main__":
    main()
