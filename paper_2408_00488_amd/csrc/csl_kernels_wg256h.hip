// The persistent MINRES solver (arXiv:2408.00488) compiled for workgroups of
// 256 threads with the FP16 split-product sine-matrix engine, namespace
// csl::wg256h.  Only problems and batches that have an axis on that engine
// use it: its extra code paths raise the register pressure of the whole
// kernel, which the other systems should not pay for in csl::wg256.
#define CSL_NT 256
#define CSL_KNS wg256h
#define CSL_SOLVE_ONLY 1
#define CSL_GEMM16 1
#include "csl_kernels.hip"
