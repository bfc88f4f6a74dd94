// The persistent MINRES solver (arXiv:2408.00488) compiled for one
// workgroup of 1024 threads per CU that holds the whole LDS, namespace
// csl::wg1024p, for 3-D systems with the FP32 preconditioner whose planes of
// the two leading axes fit in LDS: their iteration is X, the plane phase
// (tile_YP: the transforms along axes 1 and 0 of the real or imaginary part
// of one plane at a time), Z, three phases instead of five.  Sixteen waves per CU at 128 registers, as
// two workgroups of the 512-thread instances.
#define CSL_NT 1024
#define CSL_KNS wg1024p
#define CSL_SOLVE_ONLY 1
#define CSL_FFT_ONLY 1
#define CSL_PLANE 1
#define CSL_WAVES_PER_EU 4
#include "csl_kernels.hip"
