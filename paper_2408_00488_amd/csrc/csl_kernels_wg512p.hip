// The persistent MINRES solver (arXiv:2408.00488) compiled for one
// workgroup of 512 threads per CU that holds the whole LDS, namespace
// csl::wg512p, for 3-D systems with the FP64 preconditioner whose planes of
// the two leading axes fit in LDS: the plane phase (tile_YP) on one FP64
// part of a plane at a time, as csl::wg1024p does in FP32.  An FP64 plane of
// 127 x 127 points takes 126 KiB, which leaves room for the line buffers of
// eight waves only.
#define CSL_NT 512
#define CSL_KNS wg512p
#define CSL_SOLVE_ONLY 1
#define CSL_FFT_ONLY 1
#define CSL_PLANE 1
#define CSL_PLANE_F64 1
#define CSL_WAVES_PER_EU 2
#include "csl_kernels.hip"
