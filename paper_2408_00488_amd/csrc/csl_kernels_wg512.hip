// The persistent MINRES solver (arXiv:2408.00488) compiled for workgroups of
// 512 threads, namespace csl::wg512.  It holds only the solve kernel and its
// phase tiles, specialised to 2-D systems whose sine transforms all run on
// the LDS FFT: with eight waves per workgroup the FFT stages need half the
// registers per thread, so two workgroups of 512 threads (16 waves) fit a CU
// at 128 registers instead of two of 256 (8 waves) at 256.  The runtime
// chooses it for such problems and batches; everything else uses the
// 256-thread instance built from the same source.
#define CSL_NT 512
#define CSL_KNS wg512
#define CSL_SOLVE_ONLY 1
#define CSL_2D_FFT_ONLY 1
#include "csl_kernels.hip"
