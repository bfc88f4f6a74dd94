// Host-callable launch wrappers of the gfx950 kernels.  The device code is
// built six times: csl::wg256 (256-thread workgroups; every kernel),
// csl::wg256h (the 256-thread persistent solver with the FP16 split-product
// sine-matrix engine), csl::wg512 (512-thread workgroups; the persistent
// solver for 2-D systems whose transforms all run on the LDS FFT),
// csl::wg512x (the same for FFT systems of either dimension), csl::wg1024p
// (one 1024-thread workgroup per CU: the 3-D solver with the plane phase,
// FP32 preconditioner) and csl::wg512p (one 512-thread workgroup per CU: the
// same with the FP64 preconditioner).
#pragma once
#include "csl_common.hpp"

namespace csl {

// Threads per workgroup of the stand-alone and set-up kernels (wg256).
constexpr int kAuxThreads = 256;

namespace wg256 {

hipError_t upload_twiddles(const double2 *tw64, const float2 *tw32);
hipError_t launch_init(const SysDesc *dsys, int nsys, Glob *G, hipStream_t s);
hipError_t launch_solve(const SysDesc *dsys, const IOPtr *dio, IOPtr io0, int nsys,
                        const SolveParams &P, Glob *G, int grid, size_t smem, hipStream_t s);
hipError_t solve_occupancy(size_t smem, int *blocks_per_cu);
// y = A x; 3-D grids with at least 16 planes take the marching kernel.
hipError_t launch_apply_A(const SysDesc *dsys, int d, const int n[3], int M, const double2 *x,
                          double2 *y, hipStream_t s);
hipError_t launch_pinv_pass(const SysDesc *dsys, int d, int prec, int pass, int ntile, size_t smem,
                            const double2 *x, double2 *y, hipStream_t s);
hipError_t launch_adjoint(const SysDesc *dsys, int d, int M, const double2 *ytil,
                          const double2 *z, double2 *gf, double *ga, double *part, int nblk,
                          double *galpha, double *gbeta, hipStream_t s);
hipError_t launch_conj(const double2 *x, double2 *y, int M, hipStream_t s);
// Step transform of an all-at-once vector (L = 2^lg steps of M points, 8 <= L
// <= 1024): forward = DFT over the steps after the alpha^(k/L) scaling,
// inverse = its inverse.
hipError_t launch_step_transform(const double2 *x, double2 *y, int M, int lg, double alpha_c,
                                 int inverse, hipStream_t s);
// Store the descriptor h at dst (device) and fill the eigenvalue tables
// h.mu[*], h.mu_f[*] point to.
hipError_t launch_write_desc(const SysDesc &h, SysDesc *dst, hipStream_t s);
hipError_t launch_coef_stats(const SysDesc *dsys, int d, int M, double *part, int nblk,
                             double *out, hipStream_t s);

}  // namespace wg256

namespace wg512 {

hipError_t upload_twiddles(const double2 *tw64, const float2 *tw32);
hipError_t launch_solve(const SysDesc *dsys, const IOPtr *dio, IOPtr io0, int nsys,
                        const SolveParams &P, Glob *G, int grid, size_t smem, hipStream_t s);
hipError_t solve_occupancy(size_t smem, int *blocks_per_cu);

}  // namespace wg512

namespace wg256h {

hipError_t upload_twiddles(const double2 *tw64, const float2 *tw32);
hipError_t launch_solve(const SysDesc *dsys, const IOPtr *dio, IOPtr io0, int nsys,
                        const SolveParams &P, Glob *G, int grid, size_t smem, hipStream_t s);
hipError_t solve_occupancy(size_t smem, int *blocks_per_cu);

}  // namespace wg256h

namespace wg1024p {

hipError_t upload_twiddles(const double2 *tw64, const float2 *tw32);
hipError_t launch_solve(const SysDesc *dsys, const IOPtr *dio, IOPtr io0, int nsys,
                        const SolveParams &P, Glob *G, int grid, size_t smem, hipStream_t s);
hipError_t solve_occupancy(size_t smem, int *blocks_per_cu);

}  // namespace wg1024p

namespace wg512p {

hipError_t upload_twiddles(const double2 *tw64, const float2 *tw32);
hipError_t launch_solve(const SysDesc *dsys, const IOPtr *dio, IOPtr io0, int nsys,
                        const SolveParams &P, Glob *G, int grid, size_t smem, hipStream_t s);
hipError_t solve_occupancy(size_t smem, int *blocks_per_cu);

}  // namespace wg512p

namespace wg512x {

hipError_t upload_twiddles(const double2 *tw64, const float2 *tw32);
hipError_t launch_solve(const SysDesc *dsys, const IOPtr *dio, IOPtr io0, int nsys,
                        const SolveParams &P, Glob *G, int grid, size_t smem, hipStream_t s);
hipError_t solve_occupancy(size_t smem, int *blocks_per_cu);

}  // namespace wg512x

}  // namespace csl
