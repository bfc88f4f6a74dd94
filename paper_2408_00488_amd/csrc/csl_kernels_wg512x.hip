// The persistent MINRES solver (arXiv:2408.00488) compiled for workgroups of
// 512 threads for systems of either dimension whose sine transforms all run
// on the LDS FFT, namespace csl::wg512x.  It carries the 3-D phases as well
// (5 per iteration), which costs the 2-D paths a few percent of register
// allocation, so batches of 2-D systems keep csl::wg512 and this instance
// serves the FFT batches and problems that include 3-D grids.
#define CSL_NT 512
#define CSL_KNS wg512x
#define CSL_SOLVE_ONLY 1
#define CSL_FFT_ONLY 1
#include "csl_kernels.hip"
