// Host runtime and C ABI of the absolute-value preconditioned MINRES solver
// (arXiv:2408.00488): problem objects and their workspaces, tiling choices,
// the stand-alone operators, single and batched persistent solves (the batch
// optionally replayed from a captured hipGraph) and the adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "csl.h"
#include "csl_common.hpp"
#include "csl_kernels.hpp"

using namespace csl;

// Workspace of the allocation-free solve (minres_solve_noalloc): one array
// per device, loaded with the library, holding the descriptor, the control
// block, the partial sums, the eigenvalue tables and every work vector of the
// one system such a call solves.  Host code reaches it only through the
// address hipGetSymbolAddress returns on each device (the array's name is a
// host-side stand-in there).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

csl_status fail(csl_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? CSL_ERR_OOM : CSL_ERR_HIP,               \
                  std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

constexpr int kMaxDevices = 64;
bool g_tw_ready[kMaxDevices] = {false};
std::mutex g_tw_mu;   // problems may be created from several threads

// exp(-2 pi i m / TWN) in FP64 from the host sin/cos, rounded for FP32.
csl_status ensure_twiddles(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(CSL_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_tw_mu);
  if (g_tw_ready[dev]) return CSL_OK;
  std::vector<double2> t64(TWN);
  std::vector<float2> t32(TWN);
  for (int m = 0; m < TWN; ++m) {
    const double th = 2.0 * M_PI * (double)m / (double)TWN;
    t64[m] = make_double2(std::cos(th), -std::sin(th));
    t32[m] = make_float2((float)t64[m].x, (float)t64[m].y);
  }
  HIPCHK(wg256::upload_twiddles(t64.data(), t32.data()));
  HIPCHK(wg512::upload_twiddles(t64.data(), t32.data()));
  HIPCHK(wg512x::upload_twiddles(t64.data(), t32.data()));
  HIPCHK(wg256h::upload_twiddles(t64.data(), t32.data()));
  HIPCHK(wg1024p::upload_twiddles(t64.data(), t32.data()));
  HIPCHK(wg512p::upload_twiddles(t64.data(), t32.data()));
  g_tw_ready[dev] = true;
  return CSL_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int pow2floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Axes whose sine transform may run as a dense matrix product on the matrix
// cores: with n + 1 a power of two, n <= 127 keeps the n^2 products per line
// within reach of the FFT's cost, and the padded length np = n + 1 keeps the
// two LDS operands of a chunk (2 lp np elements) inside the FFT's lp L
// budget, L = 2(n + 1).  An axis with n + 1 not a power of two has no FFT
// here and must take the matrix product, for any 3 <= n <= 1022: its two
// operands take 2 np <= 2048 elements a line, the FFT's largest line, at a
// cost that grows as n^2 per line.
bool pow2_axis(int n) { return ((n + 1) & n) == 0; }
bool gemm_required(int n) { return !pow2_axis(n); }
bool gemm_eligible(int n) { return (n >= 15 && n <= 127) || gemm_required(n); }
int gemm_pad(int n) { return (n + 15) & ~15; }
// LDS elements a line of an axis takes: the FFT's odd extension 2(n + 1),
// or both GEMM operands 2 np where that is larger (n + 1 not a power of two)
int line_elems(int n) { return pow2_axis(n) ? 2 * (n + 1) : 2 * std::max(n + 1, gemm_pad(n)); }

// Orthonormal DST-I matrix entry sqrt(2/(n+1)) sin(pi (m+1)(k+1)/(n+1)),
// the angle reduced exactly in integers to [0, pi/2] first (exact zeros
// where (m+1)(k+1) is a multiple of n + 1).
double sine_entry(int n, int m, int k) {
  const int N1 = n + 1;
  int j = ((m + 1) * (k + 1)) % (2 * N1);
  double sg = 1.0;
  if (j >= N1) {
    j -= N1;
    sg = -1.0;
  }
  if (j == 0) return 0.0;
  j = std::min(j, N1 - j);
  return sg * std::sqrt(2.0 / N1) * std::sin(M_PI * (double)j / (double)N1);
}

// The matrix as the kernels take it: since W[n-1-m][k] = (-1)^k W[m][k],
// only rows m < h = ceil(n/2) are kept, split by the parity of k into two
// hp x hp blocks (hp = h rounded up to 16, zero padded):
// We[m][j] = W[m][2j], then Wo[m][j] = W[m][2j+1].
int gemm_half(int n) { return (((n + 1) / 2) + 15) & ~15; }
void sine_matrix(int n, std::vector<double> &W) {
  const int h = (n + 1) / 2, hp = gemm_half(n);
  W.assign((size_t)2 * hp * hp, 0.0);
  for (int m = 0; m < h; ++m)
    for (int j = 0; j < h; ++j) {
      if (2 * j < n) W[(size_t)m * hp + j] = sine_entry(n, m, 2 * j);
      if (2 * j + 1 < n) W[(size_t)hp * hp + (size_t)m * hp + j] = sine_entry(n, m, 2 * j + 1);
    }
}

// The persistent solver instance of a workgroup size: 1024 for 3-D systems
// with the plane phase (csl::wg1024p with the FP32 preconditioner; with the
// FP64 one, p64, csl::wg512p, whose workgroups have 512 threads), 512 for
// systems with the FFT on every axis (csl::wg512 when every system is 2-D,
// csl::wg512x otherwise) or 256 (csl::wg256h when a system has an axis on the
// FP16 split-product engine, csl::wg256 otherwise).
hipError_t solve_launch(int wg, bool all2d, bool g16, bool p64, const SysDesc *dsys, const IOPtr *dio,
                        IOPtr io0, int nsys, const SolveParams &P, Glob *G, int grid, size_t smem,
                        hipStream_t s) {
  if (wg == 1024)
    return p64 ? wg512p::launch_solve(dsys, dio, io0, nsys, P, G, grid, smem, s)
               : wg1024p::launch_solve(dsys, dio, io0, nsys, P, G, grid, smem, s);
  if (wg != 512)
    return g16 ? wg256h::launch_solve(dsys, dio, io0, nsys, P, G, grid, smem, s)
               : wg256::launch_solve(dsys, dio, io0, nsys, P, G, grid, smem, s);
  return all2d ? wg512::launch_solve(dsys, dio, io0, nsys, P, G, grid, smem, s)
               : wg512x::launch_solve(dsys, dio, io0, nsys, P, G, grid, smem, s);
}
hipError_t solve_occupancy_wg(int wg, bool all2d, bool g16, bool p64, size_t smem, int *blocks_per_cu) {
  if (wg == 1024)
    return p64 ? wg512p::solve_occupancy(smem, blocks_per_cu)
               : wg1024p::solve_occupancy(smem, blocks_per_cu);
  if (wg != 512)
    return g16 ? wg256h::solve_occupancy(smem, blocks_per_cu)
               : wg256::solve_occupancy(smem, blocks_per_cu);
  return all2d ? wg512::solve_occupancy(smem, blocks_per_cu)
               : wg512x::solve_occupancy(smem, blocks_per_cu);
}
// Some axis of the system runs on the FP16 split-product engine.
bool has_gemm16(const SysDesc &h) { return h.gemm[0] == 2 || h.gemm[1] == 2 || h.gemm[2] == 2; }
// The 512-thread solver applies: the FFT on every axis.
bool fft_everywhere(const SysDesc &h) { return !h.gemm[0] && !h.gemm[1] && !h.gemm[2]; }
bool fft_everywhere_mask(int m) { return (m & 7) == 0; }
// The plane phase applies: 3-D, the FFT on every axis, lines of at most 127
// points along the two leading axes and their plane (with the per-wave line
// buffers and the twiddles) inside the instance's LDS: 16 waves with FP32
// values (csl::wg1024p), 8 waves with FP64 values (csl::wg512p).
bool plane_ok(const SysDesc &h) {
  const int eb = h.prec ? 4 : 8, nw = h.prec ? 16 : 8;
  return h.d == 3 && fft_everywhere(h) && h.n[0] <= 127 && h.n[1] <= 127 &&
         plane_lds_bytes(h.n[0], h.n[1], h.lg[0], h.lg[1], eb, nw) <= kPlaneLdsBytes;
}
// Rewrite a tiling for the plane phase: block width one (Tq, Tv and T hold
// all real parts, then all imaginary parts, each with the plane of
// contiguous-axis index c contiguous), one K_Y chunk per part of each plane,
// no separate strided phases.
void plane_tiling(SysDesc &h) {
  h.plane = 1;
  h.lgB = 0;
  h.nchunk[K_Y] = 2 * h.n[2];
  h.nchunk[K_Y1] = h.nchunk[K_Y1I] = 0;
  int mx = 0;
  for (int k = 0; k < K_NKINDS; ++k) {
    h.ntile[k] = h.nchunk[k];
    h.cpt[k] = 1;
    mx = std::max(mx, h.ntile[k]);
  }
  h.maxtile = mx;
}
// Workgroup size for a request (0 = the larger one where allowed).
int resolve_wg(int block_threads, bool wg512_ok) {
  if (block_threads == 256) return 256;
  if (block_threads == 512) return 512;
  if (block_threads == 1024) return 1024;
  return wg512_ok ? 512 : 256;
}
bool valid_block_threads(int v) { return v == 0 || v == 256 || v == 512 || v == 1024; }

// Per-device record of the allocation-free solve's workspace (the array
// `scratch` below).
struct ScratchDev {
  char *ptr = nullptr;   // this device's copy of `scratch`
  int cus = 0;
  double wall_khz = 0.0;
};
ScratchDev g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Engine choices made by timing, per device and grid shape and precision.
typedef std::tuple<int, int, int, int, int, int> ShapeKey;   // dev, d, n0, n1, n2, prec
std::map<ShapeKey, int> g_engine_cache;                      // value: GEMM axis mask
std::mutex g_engine_mu;

}  // namespace

struct csl_problem_s {
  int device = 0;
  int cus = 0;
  double wall_khz = 0.0;
  SysDesc h{};
  SysDesc *d_desc = nullptr;
  void *mem = nullptr;
  Glob *glob = nullptr;
  double *stats = nullptr;
  double *stats_part = nullptr;
  int stats_nblk = 0;
  double2 *ytmp = nullptr;
  double2 *gtmp = nullptr;
  double *adj_part = nullptr;
  int adj_nblk = 0;
  double amin = 0, amax = 0;
  size_t smem = 0;
  int grid1 = 1;
  int tile_elems = 0;
  SysDesc h0{};          // creation-time tiling (one chunk per tile)
  size_t smem0 = 0;
  int cap = 1;           // workgroups that fill the device at this problem's LDS budget
  int tile_points = 0;   // current schedule of the problem's own solves
  int lds_bytes = 0;
  int block_threads = 256;
  bool wg512_ok = false; // the FFT on every axis: the 512-thread solver applies
  csl_grid grid{};       // creation arguments (for problem_clone)
  csl_problem_opts opts{};
  int single_te = 0;     // chunk size of the problem's own solves (0 = creation tiling)
  int part_cap = 1;      // per-tile partial-sum slots allocated
};

// Grids up to this many points may take smaller chunks for their own solves
// (problem_tune tries 512 and 1024 elements): a small system has too few
// full-size chunks to occupy the device.
constexpr int kSmallChunkPoints = 65536;
constexpr int kSmallChunkElems[2] = {512, 1024};

struct csl_batch_s {
  int device = 0;
  int count = 0;
  std::vector<csl_problem> probs;
  SysDesc *d_desc = nullptr;
  IOPtr *d_io = nullptr;
  IOPtr *h_io = nullptr;       // pinned
  IOPtr *d_io_adj = nullptr;   // (gtmp, ytmp) of every problem: the adjoint solves
  DevInfo *d_info = nullptr;
  Glob *glob = nullptr;
  void *mem = nullptr;
  size_t smem = 0;
  int grid = 1;
  SolveParams params{};
  bool use_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t copy_done = nullptr;
  bool io_valid = false;
  int grid_opt = 0;      // requested grid (0 = occupancy-filling)
  int tile_points = 0;   // current schedule
  int lds_bytes = 0;
  int block_threads = 256;
  bool wg512_ok = false; // every problem allows the 512-thread solver
  bool all2d = true;     // every problem is 2-D (the 2-D-only 512-thread instance)
  bool plane_ok = false; // every problem allows the plane phase (block_threads 1024)
                         // and all have the same preconditioner precision
  bool p64 = false;      // ... the FP64 one (the 512-thread plane instance)
  bool g16 = false;      // some problem has an axis on the FP16 split-product engine
};

struct csl_paradiag_s {
  int device = 0;
  int L = 0, lg = 0;
  int M = 0;
  double tau = 0.0, alpha_c = 0.0;
  std::vector<csl_problem> probs;   // mode j: shift D_j
  std::vector<double> dre, dim;     // D_j
  csl_batch batch = nullptr;
  void *mem = nullptr;              // Rt, Ut: L * M complex each
  double2 *rt = nullptr, *ut = nullptr;
  std::vector<const double *> fptr; // per-mode slices of rt / ut
  std::vector<double *> zptr;
};

namespace {

SolveParams make_params(double tol, int maxit, int check_true, int timeout_ms, double wall_khz) {
  SolveParams P;
  P.tol = tol > 0 ? tol : 1e-8;
  P.maxit = maxit > 0 ? maxit : 1000;
  P.check_true = check_true ? 1 : 0;
  const int tms = timeout_ms > 0 ? timeout_ms : 60000;
  P.timeout_ticks = (long long)(tms * wall_khz);
  return P;
}

// Tiling of one system: rows per tile of the FP64 row pass (K_X), of the
// preconditioner-precision row pass (K_Z), lines per tile of the strided
// passes, rows per tile of the residual pass; tile counts per phase kind and
// the LDS bytes a workgroup needs.
void choose_tiles(SysDesc &h, int tile_elems, int ldsb_min, size_t *smem_out) {
  // LDS budget per workgroup: 32 KiB unless a line of 2048 (n = 1023) needs
  // 64, or the caller asks for 64 (twice the lines per strided tile)
  int Lmax = 0;
  for (int ax = 0; ax < h.d; ++ax) Lmax = std::max(Lmax, line_elems(h.n[ax]));
  const int ldsb = (Lmax > 1024 || ldsb_min > 32768) ? 65536 : 32768;
  const int eltR = h.prec ? 8 : 16;
  const int maxeR = ldsb / eltR;
  const int maxe64 = ldsb / 16;
  const int tgt64 = tile_elems > 0 ? std::min(tile_elems, maxe64) : maxe64;
  const int tgtR = tile_elems > 0 ? std::min(tile_elems, maxeR) : maxeR;
  const int dl = h.d - 1;
  const int nlast = h.n[dl];
  const int Ll = line_elems(nlast);
  auto rows_lp = [&](int tgt, int maxe) {
    const int cap = std::max(1, std::min(64, maxe / Ll));
    return pow2floor(std::max(1, std::min(tgt / Ll, cap)));
  };
  h.lpt_x = rows_lp(tgt64, maxe64);
  h.lpt_z = rows_lp(tgtR, maxeR);
  size_t smem = std::max((size_t)h.lpt_x * Ll * 16, (size_t)h.lpt_z * Ll * eltR);
  for (int ax = 0; ax < 2; ++ax) {
    if (ax >= dl) {
      h.lpt_s[ax] = 1;
      continue;
    }
    const int L = line_elems(h.n[ax]);
    const int cap = std::max(1, std::min(64, maxeR / L));
    int want = std::max(4, tgtR / L);
    int lp = pow2floor(std::min(want, cap));
    lp = std::min(lp, pow2floor(std::max(1, nlast)) * 2);
    h.lpt_s[ax] = std::max(1, lp);
    smem = std::max(smem, (size_t)h.lpt_s[ax] * L * eltR);
  }
  // every strided pass uses the block width of the column-blocked layout
  if (h.d == 3) h.lpt_s[0] = h.lpt_s[1] = std::min(h.lpt_s[0], h.lpt_s[1]);
  h.lgB = ilog2(h.lpt_s[0]);
  h.rpt = std::max(1, tgt64 / nlast);
  for (int k = 0; k < K_NKINDS; ++k) {
    h.nchunk[k] = 0;
    h.cpt[k] = 1;
  }
  const int rows = h.rows;
  h.nchunk[K_X] = (rows + h.lpt_x - 1) / h.lpt_x;
  h.nchunk[K_Z] = (rows + h.lpt_z - 1) / h.lpt_z;
  if (h.d == 3) {
    const int nb1 = (nlast + h.lpt_s[1] - 1) / h.lpt_s[1];
    h.nchunk[K_Y1] = h.nchunk[K_Y1I] = h.n[0] * nb1;
    const int nb0 = (nlast + h.lpt_s[0] - 1) / h.lpt_s[0];
    h.nchunk[K_Y] = h.n[1] * nb0;
  } else {
    h.nchunk[K_Y] = (nlast + h.lpt_s[0] - 1) / h.lpt_s[0];
  }
  h.nchunk[K_PR] = (rows + h.rpt - 1) / h.rpt;
  for (int k = 0; k < K_NKINDS; ++k) h.ntile[k] = h.nchunk[k];
  int mx = 0;
  for (int k = 0; k < K_NKINDS; ++k) mx = std::max(mx, h.ntile[k]);
  h.maxtile = mx;
  // the 32 KiB variant stages twiddles for lengths up to 1024 only
  *smem_out = (smem <= 32768 && Lmax <= 1024 && ldsb == 32768) ? smem : 65536;
}

// Group chunks into tiles of about `points` grid points each (1 chunk per
// tile when points <= 0): fewer, larger tiles mean fewer cross-workgroup
// hand-offs (each one an L2 write-back and invalidate) per phase.
void set_tile_points(SysDesc &h, int points) {
  const int nlast = h.n[h.d - 1];
  int cpts[K_NKINDS];
  for (int k = 0; k < K_NKINDS; ++k) cpts[k] = 1;
  if (points > 0) {
    auto per = [&](int chunk_points) { return std::max(1, points / std::max(1, chunk_points)); };
    cpts[K_X] = per(h.lpt_x * nlast);
    cpts[K_Z] = per(h.lpt_z * nlast);
    cpts[K_Y] = per(h.lpt_s[0] * h.n[0]);
    if (h.d == 3) cpts[K_Y1] = cpts[K_Y1I] = per(h.lpt_s[1] * h.n[1]);
    cpts[K_PR] = per(h.rpt * nlast);
  }
  if (h.plane) cpts[K_Y] = 1;   // one part of one plane (held in LDS) per tile
  // ntile <= nchunk, so the partials buffer sized by the chunk counts (maxtile)
  // holds every tile's partial
  for (int k = 0; k < K_NKINDS; ++k) {
    h.cpt[k] = cpts[k];
    h.ntile[k] = h.nchunk[k] > 0 ? (h.nchunk[k] + cpts[k] - 1) / cpts[k] : 0;
  }
}

// A system whose status is still unset when the kernel returns was stopped
// by the time limit; one that finished keeps its own status (its solution
// is complete even when another system of the batch timed out).
csl_status info_from_device(const DevInfo &di, csl_solve_info *info) {
  csl_solve_info r;
  r.status = di.status;
  r.iters = di.iters;
  r.relres_est = di.relres_est;
  r.relres_true = di.relres_true;
  if (di.status < 0) r.status = CSL_ERR_TIMEOUT;
  if (info) *info = r;
  return (csl_status)r.status;
}

const char *status_name(csl_status st) {
  static const char *names[] = {"ok", "bad argument", "singular", "not converged",
                                "breakdown", "non-finite", "hip", "oom", "timeout"};
  return st >= 0 && st <= 8 ? names[st] : "?";
}

// Eigenvalues of the symmetric tridiagonal matrix with diagonal d and
// off-diagonal e (e[i] couples i and i + 1), ascending, by bisection on
// Sturm counts: the number of eigenvalues below x is the number of negative
// pivots of the LDL^T factorisation of T - x I.  Intervals are split until
// they hold one eigenvalue and are as narrow as the rounding allows
// (O(k^2) counts of O(k) work for k eigenvalues).
int sturm_below(const std::vector<double> &d, const std::vector<double> &e2, double x) {
  int c = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    q = d[i] - x - (i > 0 ? e2[i - 1] / q : 0.0);
    if (q == 0.0) q = -1e-300;
    c += q < 0.0;
  }
  return c;
}

void tridiag_eigenvalues(const std::vector<double> &d, const std::vector<double> &e,
                         std::vector<double> &out) {
  const int k = (int)d.size();
  out.assign(k, 0.0);
  if (k == 0) return;
  std::vector<double> e2(e.size());
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  for (size_t i = 0; i < e.size(); ++i) e2[i] = e[i] * e[i];
  const double span = std::max(std::fabs(lo), std::fabs(hi));
  lo -= 1e-12 * span + 1e-300;
  hi += 1e-12 * span + 1e-300;
  struct Iv {
    double lo, hi;
    int clo, chi;
  };
  std::vector<Iv> stack{{lo, hi, 0, k}};
  while (!stack.empty()) {
    const Iv v = stack.back();
    stack.pop_back();
    if (v.chi <= v.clo) continue;
    const double mid = 0.5 * (v.lo + v.hi);
    const double tol = 4.0 * 2.220446049250313e-16 * std::max(std::fabs(v.lo), std::fabs(v.hi));
    if (v.hi - v.lo <= tol || mid <= v.lo || mid >= v.hi) {
      for (int i = v.clo; i < v.chi; ++i) out[i] = mid;
      continue;
    }
    const int cm = std::min(std::max(sturm_below(d, e2, mid), v.clo), v.chi);
    stack.push_back({v.lo, mid, v.clo, cm});
    stack.push_back({mid, v.hi, cm, v.chi});
  }
}

// Lanczos coefficients recorded by the last solve of p (its own or within a
// batch): delta_1..delta_k, gamma_2..gamma_{k+1}.
csl_status read_lanczos(csl_problem p, std::vector<double> &delta, std::vector<double> &gamma,
                        hipStream_t s) {
  std::vector<double> buf(2 * kLanczosCap + 1);
  HIPCHK(hipMemcpyAsync(buf.data(), p->h.lz, sizeof(double) * buf.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int k = std::min(kLanczosCap, std::max(0, (int)buf[2 * kLanczosCap]));
  delta.resize(k);
  gamma.resize(k);
  for (int j = 0; j < k; ++j) {
    delta[j] = buf[2 * j];
    gamma[j] = buf[2 * j + 1];
  }
  return CSL_OK;
}

void free_problem(csl_problem p) {
  if (!p) return;
  if (p->mem) (void)hipFree(p->mem);
  delete p;
}

// P^{-1} x as its sequence of transform passes: 0 rows forward, 1 axis-1
// forward (3-D), 2 axis 0 with the mode scaling, 3 axis-1 inverse (3-D),
// 4 rows inverse.
hipError_t launch_pinv_all(csl_problem p, const double2 *x, double2 *y, hipStream_t s) {
  const SysDesc &h = p->h;
  const int nrow = (h.rows + h.lpt_z - 1) / h.lpt_z;
  const int pass[5] = {0, 1, 2, 3, 4};
  for (int k = 0; k < 5; ++k) {
    if (h.d == 2 && (pass[k] == 1 || pass[k] == 3)) continue;
    // one workgroup per LDS chunk (the solver's tiles may group chunks)
    const int nt = pass[k] == 0 || pass[k] == 4 ? nrow
                   : pass[k] == 2             ? h.nchunk[K_Y]
                   : pass[k] == 1             ? h.nchunk[K_Y1]
                                              : h.nchunk[K_Y1I];
    const hipError_t e = wg256::launch_pinv_pass(p->d_desc, h.d, h.prec, pass[k], nt, p->smem, x, y, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Schedule of a problem's own solves: the creation-time tiling with an LDS
// budget of at least `lds_bytes` and chunks grouped into tiles of
// `tile_points` points (0: about one tile per workgroup and phase, since a
// single solve has the whole device).
csl_status configure_single(csl_problem p, int tile_points, int lds_bytes, int block_threads,
                            hipStream_t s) {
  SysDesc h = p->h0;
  size_t sm = p->smem0;
  const bool plane = block_threads == 1024;
  if (plane) {
    if (!plane_ok(h))
      return fail(CSL_ERR_ARG, "block_threads 1024 (the plane phase) needs a 3-D problem with the "
                               "FFT on every axis and n0, n1 <= 127 (n0 n1 <= 16129 with FP64)");
    // the row phases on a 64 KiB line buffer, then the plane layout
    choose_tiles(h, p->single_te > 0 ? p->single_te : p->tile_elems, 65536, &sm);
    plane_tiling(h);
  } else if (p->single_te > 0) {
    choose_tiles(h, p->single_te, lds_bytes, &sm);
  } else if (lds_bytes > 32768 && p->smem0 <= 32768) {
    choose_tiles(h, p->tile_elems, lds_bytes, &sm);
  }
  // every tile of every phase owns a partial-sum slot
  if (h.maxtile > p->part_cap) return fail(CSL_ERR_ARG, "chunking exceeds the partial-sum slots");
  const int wg = resolve_wg(block_threads, p->wg512_ok);
  int bpc = 0;
  HIPCHK(solve_occupancy_wg(wg, p->h0.d == 2, has_gemm16(p->h0), p->h0.prec == 0, sm, &bpc));
  const int cap = std::max(1, bpc) * p->cus;
  const int tp = tile_points > 0 ? tile_points : (int)std::min<long long>(1 << 30, h.M / cap);
  set_tile_points(h, tp);
  int mt = 1;
  for (int k = 0; k < K_NKINDS; ++k) mt = std::max(mt, h.ntile[k]);
  HIPCHK(hipMemcpyAsync(p->d_desc, &h, sizeof(SysDesc), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  p->h = h;
  p->smem = sm;
  p->cap = cap;
  p->grid1 = std::max(1, std::min(mt, cap));
  p->tile_points = tile_points;
  p->lds_bytes = sm <= 32768 ? 32768 : 65536;
  p->block_threads = wg;
  return CSL_OK;
}

// Choose the matrix-core axes by timing the problem's own solve: a few
// MINRES iterations (fixed count, constant right-hand side) of the
// persistent solver with every admissible subset of the eligible axes (one
// that holds every axis without an FFT, n + 1 not a power of two), each
// with its default single-solve schedule and the workgroup size it allows
// (the 512-thread solver needs the FFT on both axes of a 2-D grid); the
// fastest is kept, the FFT winning anything within 2%.  Timing the solver
// itself, one launch per solve, charges each engine with what it costs in
// the iteration (transform, staging, occupancy) rather than in stand-alone
// transform passes.  Runs on p's workspaces; the caller then sets the
// chosen engines and rewrites p's descriptor and schedule.
csl_status tune_engines(csl_problem p, int elig, int req, hipStream_t s, int *best_mask) {
  *best_mask = req;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(CSL_ERR_HIP, "hipEventCreate failed");
  }
  const SysDesc h_in = p->h;
  const size_t smem_in = p->smem;
  // f: every byte 0x3f, i.e. every real and imaginary part 4.8e-4
  hipError_t err = hipMemsetAsync(p->gtmp, 0x3f, sizeof(double2) * (size_t)h_in.M, s);
  const SolveParams P = make_params(1e-300, 6, 0, 0, p->wall_khz);
  const IOPtr io0{p->gtmp, p->ytmp};
  const int reps = 3;
  float best = INFINITY;
  csl_status st = CSL_OK;
  for (int mask = 0; mask < 8 && err == hipSuccess && st == CSL_OK; ++mask) {
    if ((mask & ~elig) || (mask & req) != req) continue;
    SysDesc h = h_in;
    for (int ax = 0; ax < 3; ++ax) h.gemm[ax] = (mask >> ax) & 1;
    p->h = h;
    p->h0 = h;
    p->smem0 = smem_in;
    p->wg512_ok = fft_everywhere(h);
    st = configure_single(p, 0, 0, 0, s);
    if (st != CSL_OK) break;
    for (int r = 0; r <= reps && err == hipSuccess; ++r) {
      if (r == 1) err = hipEventRecord(e0, s);   // the first solve is a warm-up
      if (err == hipSuccess) err = wg256::launch_init(p->d_desc, 1, p->glob, s);
      if (err == hipSuccess)
        err = solve_launch(p->block_threads, h.d == 2, has_gemm16(h), h.prec == 0, p->d_desc, nullptr,
                           io0, 1,
                           P, p->glob,
                           p->grid1,
                           p->smem, s);
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && (mask == req ? ms < best : ms < 0.98f * best)) {
      best = ms;
      *best_mask = mask;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->h = h_in;
  p->smem = smem_in;
  if (st != CSL_OK) return st;
  if (err != hipSuccess) return fail(CSL_ERR_HIP, std::string("engine timing: ") + hipGetErrorString(err));
  return CSL_OK;
}

// Schedule of a batch: descriptor copies tiled for `tile_points` grid points
// per tile and an LDS budget of at least `lds_bytes`, the grid, and (if
// asked) the captured graph of one solve.  Called at creation and by the
// tuner.
csl_status configure_batch(csl_batch b, int tile_points, int lds_bytes, int block_threads,
                           bool graph) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  std::vector<SysDesc> descs(b->count);
  size_t smem = 0;
  const bool plane = resolve_wg(block_threads, b->wg512_ok) == 1024;
  for (int i = 0; i < b->count; ++i) {
    const csl_problem p = b->probs[i];
    descs[i] = p->h0;
    size_t sm = p->smem0;
    if (plane) {
      // the row phases on a 64 KiB line buffer, then the plane layout
      choose_tiles(descs[i], p->tile_elems, 65536, &sm);
      plane_tiling(descs[i]);
      if (descs[i].maxtile > p->part_cap)
        return fail(CSL_ERR_ARG, "chunking exceeds the partial-sum slots");
    } else if (lds_bytes > 32768 && p->smem0 <= 32768) {
      // a larger budget only lengthens the chunks: chunk counts (and with
      // them the partial-sum slots each problem allocated) can only shrink
      choose_tiles(descs[i], p->tile_elems, lds_bytes, &sm);
    }
    descs[i].info = b->d_info + i;
    set_tile_points(descs[i], tile_points);
    smem = std::max(smem, sm);
  }
  HIPCHK(hipMemcpy(b->d_desc, descs.data(), sizeof(SysDesc) * b->count, hipMemcpyHostToDevice));
  b->smem = smem;
  b->tile_points = tile_points;
  b->lds_bytes = smem <= 32768 ? 32768 : 65536;
  b->block_threads = resolve_wg(block_threads, b->wg512_ok);
  int bpc = 0;
  HIPCHK(solve_occupancy_wg(b->block_threads, b->all2d, b->g16, b->p64, smem, &bpc));
  // tiles are claimed dynamically, so a full-occupancy grid keeps every CU
  // busy whatever the mix of systems
  const int cap = std::max(1, bpc) * b->probs[0]->cus;
  b->grid = std::max(1, b->grid_opt > 0 ? b->grid_opt : cap);
  if (!graph) return CSL_OK;
  hipStream_t cs;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    ok = wg256::launch_init(b->d_desc, b->count, b->glob, cs) == hipSuccess;
    IOPtr none{nullptr, nullptr};
    ok = ok && solve_launch(b->block_threads, b->all2d, b->g16, b->p64, b->d_desc, b->d_io, none, b->count,
                            b->params,
                            b->glob, b->grid, b->smem, cs) == hipSuccess;
    hipGraph_t g = nullptr;
    const bool ended = hipStreamEndCapture(cs, &g) == hipSuccess;
    ok = ok && ended && g;
    if (ok) ok = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) == hipSuccess;
    b->graph = g;
  }
  (void)hipStreamDestroy(cs);
  if (!ok) return fail(CSL_ERR_HIP, "hipGraph capture of the batched solve failed");
  return CSL_OK;
}

// Geometry of a system from the caller's grid: sizes, strides, mesh widths,
// FFT lengths (the rest of the descriptor is left as it is).
csl_status grid_desc(const csl_grid *grid, SysDesc &h) {
  if (grid->dim != 2 && grid->dim != 3) return fail(CSL_ERR_ARG, "dim must be 2 or 3");
  h.d = grid->dim;
  long long M = 1;
  for (int ax = 0; ax < 3; ++ax) {
    if (ax < h.d) {
      const int n = grid->n[ax];
      if (n < 3 || n > TWN / 2 - 1)
        return fail(CSL_ERR_ARG, "n[" + std::to_string(ax) + "] must be between 3 and 1023");
      const double len = grid->length[ax] > 0 ? grid->length[ax] : 1.0;
      if (!std::isfinite(len)) return fail(CSL_ERR_ARG, "length must be finite");
      const double hh = len / (n + 1);
      h.n[ax] = n;
      h.h2[ax] = 1.0 / (hh * hh);
      h.lg[ax] = ilog2(2 * (n + 1));
      M *= n;
    } else {
      h.n[ax] = 1;
      h.h2[ax] = 0.0;
      h.lg[ax] = 0;
    }
  }
  if (M > (1ll << 30)) return fail(CSL_ERR_ARG, "grid too large");
  h.M = (int)M;
  h.st[h.d - 1] = 1;
  for (int ax = h.d - 2; ax >= 0; --ax) h.st[ax] = h.st[ax + 1] * h.n[ax + 1];
  h.rows = h.M / h.n[h.d - 1];
  return CSL_OK;
}

// The singularity test of P (beta = 0 and abar * mu + alpha = 0 for some mode
// k): true if min_k |abar mu_k + alpha| is 0 or negligible against the
// largest.  mu: the per-axis tables back to back (n0 + n1 + n2 entries).
bool preconditioner_singular(const SysDesc &h, const std::vector<double> &mu, double abar,
                             double alpha, double beta) {
  if (beta != 0.0) return false;
  double mn = INFINITY, mxv = 0.0;
  const int n0 = h.n[0], n1 = h.n[1], n2 = h.d == 3 ? h.n[2] : 1;
  const double *m0 = mu.data(), *m1 = mu.data() + h.n[0], *m2 = mu.data() + h.n[0] + h.n[1];
  for (int i = 0; i < n0; ++i)
    for (int j = 0; j < n1; ++j)
      for (int k = 0; k < n2; ++k) {
        const double lam = m0[i] + m1[j] + (h.d == 3 ? m2[k] : 0.0);
        const double v = std::fabs(abar * lam + alpha);
        mn = std::min(mn, v);
        mxv = std::max(mxv, v);
      }
  return mn <= 1e-300 || mn <= 1e-14 * mxv;
}

}  // namespace

extern "C" {

int csl_version(void) { return 200; }

const char *csl_last_error(void) { return g_err.c_str(); }

// forced_mask >= 0: the matrix-core axes are given (problem_clone), no
// engine selection
static csl_status create_problem_impl(const csl_grid *grid, const double *a_nodal, double alpha,
                                      double beta, const csl_problem_opts *opts, hipStream_t s,
                                      csl_problem *out, int forced_mask) {
  if (!out) return fail(CSL_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!grid || !a_nodal) return fail(CSL_ERR_ARG, "grid or coefficient is NULL");
  if (!std::isfinite(alpha) || !std::isfinite(beta))
    return fail(CSL_ERR_ARG, "shift must be finite");
  csl_problem_opts o{};
  o.abar_rule = CSL_ABAR_MEAN;
  o.pinv_prec = CSL_PREC_FP64;
  if (opts) o = *opts;
  if (o.abar_rule < 0 || o.abar_rule > 2) return fail(CSL_ERR_ARG, "unknown abar rule");
  if (o.pinv_prec != CSL_PREC_FP64 && o.pinv_prec != CSL_PREC_FP32)
    return fail(CSL_ERR_ARG, "unknown preconditioner precision");
  if (o.abar_rule == CSL_ABAR_GIVEN && !(o.abar > 0 && std::isfinite(o.abar)))
    return fail(CSL_ERR_ARG, "given abar must be finite and positive");
  if (o.dst_engine < CSL_DST_AUTO || o.dst_engine > CSL_DST_GEMM16)
    return fail(CSL_ERR_ARG, "unknown sine-transform engine");
  if (o.dst_engine == CSL_DST_GEMM16 && o.pinv_prec != CSL_PREC_FP32)
    return fail(CSL_ERR_ARG, "the FP16 split-product engine needs the FP32 preconditioner");

  SysDesc h{};
  {
    const csl_status st = grid_desc(grid, h);
    if (st != CSL_OK) return st;
  }
  h.prec = o.pinv_prec;
  h.alpha = alpha;
  h.beta = beta;

  csl_problem p = new csl_problem_s();
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete p;
    return fail(CSL_ERR_HIP, "hipGetDevice failed");
  }
  p->device = dev;
  {
    csl_status st = ensure_twiddles(dev);
    if (st != CSL_OK) {
      delete p;
      return st;
    }
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete p;
    return fail(CSL_ERR_HIP, "hipGetDeviceProperties failed");
  }
  p->cus = prop.multiProcessorCount;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  p->wall_khz = (double)khz;

  if (o.tile_elems < 0) {
    delete p;
    return fail(CSL_ERR_ARG, "tile_elems must be >= 0");
  }
  choose_tiles(h, o.tile_elems, 0, &p->smem);
  p->tile_elems = o.tile_elems;
  p->stats_nblk = std::min(1024, (h.M + kAuxThreads - 1) / kAuxThreads);
  p->adj_nblk = std::min(1024, (h.M + kAuxThreads - 1) / kAuxThreads);

  // one allocation for the coefficient copy, tables and workspaces
  const size_t vec = align256(sizeof(double2) * (size_t)h.M);
  // column-blocked vectors: rows x ceil(n_last / B) B entries, B <= 64
  const size_t Mb = (size_t)h.rows * (size_t)(h.n[h.d - 1] + 63);
  const size_t vecb = align256(sizeof(double2) * Mb);
  const size_t tsz = align256(Mb * (h.prec ? 8 : 16));
  const int nmu = h.n[0] + h.n[1] + h.n[2];
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o2 = off;
    off += align256(bytes);
    return o2;
  };
  const size_t o_a = take(sizeof(double) * h.M);
  const size_t o_mu = take(sizeof(double) * nmu);
  const size_t o_muf = take(sizeof(float) * nmu);
  size_t o_v[7];
  for (int i = 0; i < 7; ++i) o_v[i] = take(i < 3 ? vecb : vec);   // Tq, Tv0, Tv1 blocked
  const size_t o_t = take(tsz);
  // partial-sum slots: the creation-time chunking, and on small grids the
  // smallest chunks problem_tune may choose for the problem's own solves
  int part_cap = std::max(1, h.maxtile);
  // the plane phase's tiling (3-D): one tile per part (real, imaginary) of
  // each plane of the contiguous axis, its row phases on chunks no smaller
  // than these
  if (h.d == 3) part_cap = std::max(part_cap, 2 * h.n[2]);
  if (h.M <= kSmallChunkPoints) {
    SysDesc t = h;
    size_t sm_t = 0;
    choose_tiles(t, kSmallChunkElems[0], 0, &sm_t);
    part_cap = std::max(part_cap, t.maxtile);
  }
  const size_t o_part = take(sizeof(double) * part_cap);
  const size_t o_ctl = take(sizeof(Ctl));
  const size_t o_info = take(sizeof(DevInfo));
  const size_t o_glob = take(sizeof(Glob));
  const size_t o_desc = take(sizeof(SysDesc));
  const size_t o_stats = take(sizeof(double) * 4);
  const size_t o_spart = take(sizeof(double) * 4 * p->stats_nblk);
  const size_t o_ytmp = take(vec);
  const size_t o_gtmp = take(vec);
  const size_t o_apart = take(sizeof(double) * 2 * p->adj_nblk);
  const size_t o_lz = take(sizeof(double) * (2 * kLanczosCap + 1));
  size_t o_w[3] = {0, 0, 0}, o_wf[3] = {0, 0, 0}, o_wh[3] = {0, 0, 0};
  int elig = 0, req = 0;
  const bool g16 = o.dst_engine == CSL_DST_GEMM16;
  for (int ax = 0; ax < h.d; ++ax) {
    if (!gemm_eligible(h.n[ax])) continue;
    elig |= 1 << ax;
    if (gemm_required(h.n[ax])) req |= 1 << ax;
    const size_t wsz = (size_t)2 * gemm_half(h.n[ax]) * gemm_half(h.n[ax]);
    o_w[ax] = take(sizeof(double) * wsz);
    o_wf[ax] = take(sizeof(float) * wsz);
    if (g16) o_wh[ax] = take(sizeof(_Float16) * 2 * wsz);   // high and low parts
  }
  hipError_t e = hipMalloc(&p->mem, off);
  if (e != hipSuccess) {
    delete p;
    return fail(e == hipErrorOutOfMemory ? CSL_ERR_OOM : CSL_ERR_HIP,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  char *base = (char *)p->mem;
  double *d_a = (double *)(base + o_a);
  double *d_mu = (double *)(base + o_mu);
  float *d_muf = (float *)(base + o_muf);
  h.a = d_a;
  h.Tq = (double2 *)(base + o_v[0]);
  h.Tv[0] = (double2 *)(base + o_v[1]);
  h.Tv[1] = (double2 *)(base + o_v[2]);
  h.Z[0] = (double2 *)(base + o_v[3]);
  h.Z[1] = (double2 *)(base + o_v[4]);
  h.W[0] = (double2 *)(base + o_v[5]);
  h.W[1] = (double2 *)(base + o_v[6]);
  h.T = base + o_t;
  h.part = (double *)(base + o_part);
  h.ctl = (Ctl *)(base + o_ctl);
  h.info = (DevInfo *)(base + o_info);
  p->glob = (Glob *)(base + o_glob);
  p->part_cap = part_cap;
  p->d_desc = (SysDesc *)(base + o_desc);
  p->stats = (double *)(base + o_stats);
  p->stats_part = (double *)(base + o_spart);
  p->ytmp = (double2 *)(base + o_ytmp);
  p->gtmp = (double2 *)(base + o_gtmp);
  p->adj_part = (double *)(base + o_apart);
  h.lz = (double *)(base + o_lz);
  for (int ax = 0; ax < 3; ++ax) {
    h.gemm[ax] = 0;
    h.Wm[ax] = (elig >> ax & 1) ? (const double *)(base + o_w[ax]) : nullptr;
    h.Wmf[ax] = (elig >> ax & 1) ? (const float *)(base + o_wf[ax]) : nullptr;
    h.Wmh[ax] = (g16 && (elig >> ax & 1)) ? (const void *)(base + o_wh[ax]) : nullptr;
  }

  // per-axis eigenvalues of L: (4/h^2) sin^2(k pi / (2(n+1)))
  std::vector<double> mu(nmu);
  std::vector<float> muf(nmu);
  int mo = 0;
  for (int ax = 0; ax < 3; ++ax) {
    h.mu[ax] = d_mu + mo;
    h.mu_f[ax] = d_muf + mo;
    const int n = h.n[ax];
    for (int k = 1; k <= n; ++k) {
      const double sv = std::sin((double)k * M_PI / (2.0 * (n + 1)));
      mu[mo + k - 1] = ax < h.d ? 4.0 * h.h2[ax] * sv * sv : 0.0;
      muf[mo + k - 1] = (float)mu[mo + k - 1];
    }
    mo += n;
  }
  double st4[4];
#define PCHK(call)                                                                   \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      free_problem(p);                                                               \
      return fail(CSL_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    }                                                                                \
  } while (0)
  PCHK(hipMemcpyAsync(d_a, a_nodal, sizeof(double) * h.M, hipMemcpyDeviceToDevice, s));
  PCHK(hipMemsetAsync(h.lz, 0, sizeof(double) * (2 * kLanczosCap + 1), s));
  PCHK(hipMemcpyAsync(d_mu, mu.data(), sizeof(double) * nmu, hipMemcpyHostToDevice, s));
  PCHK(hipMemcpyAsync(d_muf, muf.data(), sizeof(float) * nmu, hipMemcpyHostToDevice, s));
  std::vector<double> Wt[3];
  std::vector<float> Wtf[3];
  std::vector<_Float16> Wth[3];
  for (int ax = 0; ax < h.d; ++ax) {
    if (!(elig >> ax & 1)) continue;
    sine_matrix(h.n[ax], Wt[ax]);
    Wtf[ax].resize(Wt[ax].size());
    for (size_t i = 0; i < Wt[ax].size(); ++i) Wtf[ax][i] = (float)Wt[ax][i];
    PCHK(hipMemcpyAsync((void *)h.Wm[ax], Wt[ax].data(), sizeof(double) * Wt[ax].size(),
                        hipMemcpyHostToDevice, s));
    PCHK(hipMemcpyAsync((void *)h.Wmf[ax], Wtf[ax].data(), sizeof(float) * Wtf[ax].size(),
                        hipMemcpyHostToDevice, s));
    if (g16) {
      // 2^kGemm16Shift W split into FP16 high and low parts: both even / odd
      // blocks of the high part, then both of the low part
      const size_t wsz = Wt[ax].size();
      Wth[ax].resize(2 * wsz);
      for (size_t i = 0; i < wsz; ++i) {
        const double w = std::ldexp(Wt[ax][i], kGemm16Shift);
        const _Float16 hi = (_Float16)w;
        Wth[ax][i] = hi;
        Wth[ax][wsz + i] = (_Float16)(w - (double)hi);
      }
      PCHK(hipMemcpyAsync((void *)h.Wmh[ax], Wth[ax].data(), sizeof(_Float16) * Wth[ax].size(),
                          hipMemcpyHostToDevice, s));
    }
  }
  PCHK(hipMemcpyAsync(p->d_desc, &h, sizeof(SysDesc), hipMemcpyHostToDevice, s));
  PCHK(wg256::launch_coef_stats(p->d_desc, h.d, h.M, p->stats_part, p->stats_nblk, p->stats, s));
  PCHK(hipMemcpyAsync(st4, p->stats, sizeof(st4), hipMemcpyDeviceToHost, s));
  PCHK(hipStreamSynchronize(s));
  if (st4[3] != 0.0) {
    free_problem(p);
    return fail(CSL_ERR_ARG, "coefficient samples must be finite and positive");
  }
  p->amin = st4[1];
  p->amax = st4[2];
  double abar = 0.0;
  if (o.abar_rule == CSL_ABAR_MEAN) abar = st4[0] / (double)h.M;
  else if (o.abar_rule == CSL_ABAR_GEOMEAN) abar = std::sqrt(st4[1] * st4[2]);
  else abar = o.abar;
  h.abar = abar;
  h.abar_f = (float)abar;
  h.alpha_f = (float)alpha;
  h.beta_f = (float)beta;
  // P is singular only if beta = 0 and abar * mu_sum + alpha = 0 for some mode
  if (preconditioner_singular(h, mu, abar, alpha, beta)) {
    free_problem(p);
    return fail(CSL_ERR_SINGULAR, "preconditioner is singular: beta = 0 and "
                                  "abar*mu + alpha = 0 for some mode");
  }
  p->h = h;
  PCHK(hipMemcpyAsync(p->d_desc, &p->h, sizeof(SysDesc), hipMemcpyHostToDevice, s));
  PCHK(hipStreamSynchronize(s));
  if (o.dst_engine == CSL_DST_FFT && req) {
    free_problem(p);
    return fail(CSL_ERR_ARG, "an axis with n + 1 not a power of two needs the dense sine-matrix "
                             "transform (dst_engine auto or gemm)");
  }
  int mask = req;
  if (forced_mask >= 0) {
    mask = forced_mask & elig;
  } else if (o.dst_engine == CSL_DST_GEMM || g16) {
    mask = elig;
  } else if (o.dst_engine == CSL_DST_AUTO && elig != req) {
    const ShapeKey key{dev, h.d, h.n[0], h.n[1], h.n[2], h.prec};
    bool have = false;
    {
      std::lock_guard<std::mutex> lk(g_engine_mu);
      auto it = g_engine_cache.find(key);
      if (it != g_engine_cache.end()) {
        mask = it->second;
        have = true;
      }
    }
    if (!have) {
      const csl_status st = tune_engines(p, elig, req, s, &mask);
      if (st != CSL_OK) {
        free_problem(p);
        return st;
      }
      std::lock_guard<std::mutex> lk(g_engine_mu);
      g_engine_cache[key] = mask;
    }
  }
  for (int ax = 0; ax < 3; ++ax) p->h.gemm[ax] = ((mask >> ax) & 1) ? (g16 ? 2 : 1) : 0;
  PCHK(hipMemcpyAsync(p->d_desc, &p->h, sizeof(SysDesc), hipMemcpyHostToDevice, s));
  PCHK(hipStreamSynchronize(s));
  p->h0 = p->h;
  p->smem0 = p->smem;
  p->wg512_ok = fft_everywhere(p->h);
  {
    const csl_status st = configure_single(p, 0, 0, 0, s);
    if (st != CSL_OK) {
      free_problem(p);
      return st;
    }
  }
#undef PCHK
  p->grid = *grid;
  p->opts = o;
  *out = p;
  return CSL_OK;
}

csl_status create_problem(const csl_grid *grid, const double *a_nodal, double alpha, double beta,
                          const csl_problem_opts *opts, hipStream_t s, csl_problem *out) {
  return create_problem_impl(grid, a_nodal, alpha, beta, opts, s, out, -1);
}

csl_status problem_clone(csl_problem p, hipStream_t s, csl_problem *out) {
  if (!out) return fail(CSL_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!p) return fail(CSL_ERR_ARG, "problem is NULL");
  csl_problem_opts o = p->opts;
  o.abar_rule = CSL_ABAR_GIVEN;   // the same abar, whichever rule produced it
  o.abar = p->h.abar;
  int mask = 0;
  for (int ax = 0; ax < 3; ++ax) mask |= (p->h.gemm[ax] ? 1 : 0) << ax;
  csl_problem q = nullptr;
  csl_status st = create_problem_impl(&p->grid, p->h.a, p->h.alpha, p->h.beta, &o, s, &q, mask);
  if (st != CSL_OK) return st;
  q->single_te = p->single_te;
  st = configure_single(q, p->tile_points, p->lds_bytes, p->block_threads, s);
  if (st != CSL_OK) {
    free_problem(q);
    return st;
  }
  *out = q;
  return CSL_OK;
}

csl_status problem_lanczos(csl_problem p, double *delta, double *gamma, int cap, int *count,
                           hipStream_t s) {
  if (!p || !count || cap < 0 || (cap > 0 && (!delta || !gamma)))
    return fail(CSL_ERR_ARG, "NULL argument or negative capacity");
  std::vector<double> d, g;
  const csl_status st = read_lanczos(p, d, g, s);
  if (st != CSL_OK) return st;
  *count = (int)d.size();
  for (int j = 0; j < std::min(cap, (int)d.size()); ++j) {
    delta[j] = d[j];
    gamma[j] = g[j];
  }
  return CSL_OK;
}

csl_status csl_tridiagonal_eigenvalues(const double *d, const double *e, int k, double *theta) {
  if (k < 0 || (k > 0 && (!d || !theta)) || (k > 1 && !e))
    return fail(CSL_ERR_ARG, "NULL argument or negative size");
  std::vector<double> dv(d, d + k), ev, th;
  if (k > 1) ev.assign(e, e + (k - 1));
  for (int i = 0; i < k; ++i)
    if (!std::isfinite(dv[i]) || (i + 1 < k && !std::isfinite(ev[i])))
      return fail(CSL_ERR_ARG, "entries must be finite");
  tridiag_eigenvalues(dv, ev, th);
  for (int i = 0; i < k; ++i) theta[i] = th[i];
  return CSL_OK;
}

csl_status problem_ritz(csl_problem p, double *theta, int cap, int *count, hipStream_t s) {
  if (!p || !count || cap < 0 || (cap > 0 && !theta))
    return fail(CSL_ERR_ARG, "NULL argument or negative capacity");
  std::vector<double> d, g, th;
  const csl_status st = read_lanczos(p, d, g, s);
  if (st != CSL_OK) return st;
  if (!d.empty()) g.resize(d.size() - 1);   // the last gamma couples to step k + 1
  tridiag_eigenvalues(d, g, th);
  *count = (int)th.size();
  for (int j = 0; j < std::min(cap, (int)th.size()); ++j) theta[j] = th[j];
  return CSL_OK;
}

csl_status destroy_problem(csl_problem p) {
  if (!p) return fail(CSL_ERR_ARG, "problem is NULL");
  free_problem(p);
  return CSL_OK;
}

csl_status problem_info(csl_problem p, double *abar, double *a_min, double *a_max) {
  if (!p) return fail(CSL_ERR_ARG, "problem is NULL");
  if (abar) *abar = p->h.abar;
  if (a_min) *a_min = p->amin;
  if (a_max) *a_max = p->amax;
  return CSL_OK;
}

csl_status problem_dst_engines(csl_problem p, int engines[3]) {
  if (!p || !engines) return fail(CSL_ERR_ARG, "NULL argument");
  for (int ax = 0; ax < 3; ++ax)
    engines[ax] = p->h.gemm[ax] == 2 ? CSL_DST_GEMM16 : (p->h.gemm[ax] ? CSL_DST_GEMM : CSL_DST_FFT);
  return CSL_OK;
}

csl_status apply_A(csl_problem p, const double *x, double *y, hipStream_t s) {
  if (!p || !x || !y) return fail(CSL_ERR_ARG, "NULL argument");
  if (x == y) return fail(CSL_ERR_ARG, "apply_A: x and y must not alias");
  HIPCHK(wg256::launch_apply_A(p->d_desc, p->h.d, p->h.n, p->h.M, (const double2 *)x,
                               (double2 *)y, s));
  return CSL_OK;
}

csl_status apply_Pinv(csl_problem p, const double *x, double *y, hipStream_t s) {
  if (!p || !x || !y) return fail(CSL_ERR_ARG, "NULL argument");
  HIPCHK(launch_pinv_all(p, (const double2 *)x, (double2 *)y, s));
  return CSL_OK;
}

static csl_status run_single(csl_problem p, const double2 *f, double2 *x, const SolveParams &P,
                             hipStream_t s) {
  HIPCHK(wg256::launch_init(p->d_desc, 1, p->glob, s));
  IOPtr io0{f, x};
  HIPCHK(solve_launch(p->block_threads, p->h.d == 2, has_gemm16(p->h), p->h.prec == 0, p->d_desc,
                      nullptr, io0, 1,
                      P, p->glob,
                      p->grid1, p->smem,
                      s));
  return CSL_OK;
}

static csl_status fetch_single_info(csl_problem p, csl_solve_info *info, hipStream_t s) {
  DevInfo di;
  HIPCHK(hipMemcpyAsync(&di, p->h.info, sizeof(di), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const csl_status st = info_from_device(di, info);
  if (st != CSL_OK) g_err = std::string("solve ended with status: ") + status_name(st);
  return st;
}

static csl_status check_solve_opts(const csl_solve_opts &o) {
  if (o.maxit > 16000000) return fail(CSL_ERR_ARG, "maxit too large");
  if (!std::isfinite(o.tol)) return fail(CSL_ERR_ARG, "tol must be finite");
  return CSL_OK;
}

csl_status minres_solve(csl_problem p, const double *f, double *z, const csl_solve_opts *opts,
                        csl_solve_info *info, hipStream_t s) {
  if (!p || !f || !z) return fail(CSL_ERR_ARG, "NULL argument");
  if (f == z) return fail(CSL_ERR_ARG, "minres_solve: f and z must not alias");
  csl_solve_opts o{};
  if (opts) o = *opts;
  if (check_solve_opts(o) != CSL_OK) return CSL_ERR_ARG;
  const SolveParams P = make_params(o.tol, o.maxit, o.check_true_residual, o.timeout_ms, p->wall_khz);
  csl_status st = run_single(p, (const double2 *)f, (double2 *)z, P, s);
  if (st != CSL_OK) return st;
  if (!info) return CSL_OK;
  return fetch_single_info(p, info, s);
}

// One-shot solve without a problem handle and without any allocation: the
// descriptor, control block, partial sums, eigenvalue tables and work vectors
// of the system live in this device's `scratch` array, the coefficient is
// read from the caller's a_nodal.  The set-up of create_problem (coefficient
// check, abar, singularity test, tiling) runs on every call; the solve is
// minres_solve's persistent kernel.
csl_status minres_solve_noalloc(const csl_grid *grid, const double *a_nodal, double alpha,
                                double beta, const csl_problem_opts *popts, const double *f,
                                double *z, const csl_solve_opts *sopts, csl_solve_info *info,
                                hipStream_t s) {
  if (!grid || !a_nodal || !f || !z) return fail(CSL_ERR_ARG, "NULL argument");
  if (f == z) return fail(CSL_ERR_ARG, "minres_solve_noalloc: f and z must not alias");
  if (!std::isfinite(alpha) || !std::isfinite(beta))
    return fail(CSL_ERR_ARG, "shift must be finite");
  csl_problem_opts o{};
  o.abar_rule = CSL_ABAR_MEAN;
  o.pinv_prec = CSL_PREC_FP64;
  if (popts) o = *popts;
  if (o.abar_rule < 0 || o.abar_rule > 2) return fail(CSL_ERR_ARG, "unknown abar rule");
  if (o.pinv_prec != CSL_PREC_FP64 && o.pinv_prec != CSL_PREC_FP32)
    return fail(CSL_ERR_ARG, "unknown preconditioner precision");
  if (o.abar_rule == CSL_ABAR_GIVEN && !(o.abar > 0 && std::isfinite(o.abar)))
    return fail(CSL_ERR_ARG, "given abar must be finite and positive");
  if (o.tile_elems < 0) return fail(CSL_ERR_ARG, "tile_elems must be >= 0");
  if (o.dst_engine != CSL_DST_AUTO && o.dst_engine != CSL_DST_FFT)
    return fail(CSL_ERR_ARG, "minres_solve_noalloc runs the FFT engine only");
  csl_solve_opts so{};
  if (sopts) so = *sopts;
  if (check_solve_opts(so) != CSL_OK) return CSL_ERR_ARG;
  SysDesc h{};
  {
    const csl_status st = grid_desc(grid, h);
    if (st != CSL_OK) return st;
  }
  for (int ax = 0; ax < h.d; ++ax)
    if (!pow2_axis(h.n[ax]))
      return fail(CSL_ERR_ARG, "minres_solve_noalloc needs n + 1 a power of two on every axis");
  h.prec = o.pinv_prec;
  h.alpha = alpha;
  h.beta = beta;
  h.alpha_f = (float)alpha;
  h.beta_f = (float)beta;
  size_t smem = 0;
  choose_tiles(h, o.tile_elems, 0, &smem);

  // layout of the workspace, as create_problem's allocation without the
  // coefficient copy, the adjoint buffers and the sine matrices
  const int stats_nblk = std::min(1024, (h.M + kAuxThreads - 1) / kAuxThreads);
  const size_t vec = align256(sizeof(double2) * (size_t)h.M);
  const size_t Mb = (size_t)h.rows * (size_t)(h.n[h.d - 1] + 63);
  const size_t vecb = align256(sizeof(double2) * Mb);
  const size_t tsz = align256(Mb * (h.prec ? 8 : 16));
  const int nmu = h.n[0] + h.n[1] + h.n[2];
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o2 = off;
    off += align256(bytes);
    return o2;
  };
  const size_t o_desc = take(sizeof(SysDesc));
  const size_t o_ctl = take(sizeof(Ctl));
  const size_t o_info = take(sizeof(DevInfo));
  const size_t o_glob = take(sizeof(Glob));
  const size_t o_stats = take(sizeof(double) * 4);
  const size_t o_spart = take(sizeof(double) * 4 * stats_nblk);
  const size_t o_part = take(sizeof(double) * std::max(1, h.maxtile));
  const size_t o_lz = take(sizeof(double) * (2 * kLanczosCap + 1));
  const size_t o_mu = take(sizeof(double) * nmu);
  const size_t o_muf = take(sizeof(float) * nmu);
  size_t o_v[7];
  for (int i = 0; i < 7; ++i) o_v[i] = take(i < 3 ? vecb : vec);   // Tq, Tv0, Tv1 blocked
  const size_t o_t = take(tsz);
  if (off > kScratchBytes)
    return fail(CSL_ERR_ARG, "minres_solve_noalloc: the grid needs " + std::to_string(off) +
                                 " bytes of workspace, more than its " +
                                 std::to_string(kScratchBytes) + "-byte limit");

  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CSL_ERR_ARG, "device index out of range");
  {
    const csl_status st = ensure_twiddles(dev);
    if (st != CSL_OK) return st;
  }
  ScratchDev sd;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchDev &e = g_scratch[dev];
    if (!e.ptr) {
      void *ptr = nullptr;
      HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
      hipDeviceProp_t prop;
      HIPCHK(hipGetDeviceProperties(&prop, dev));
      int khz = 0;
      if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
          khz <= 0)
        khz = 100000;
      e.cus = prop.multiProcessorCount;
      e.wall_khz = (double)khz;
      e.ptr = (char *)ptr;
    }
    sd = e;
  }
  char *base = sd.ptr;
  SysDesc *d_desc = (SysDesc *)(base + o_desc);
  Glob *glob = (Glob *)(base + o_glob);
  double *stats = (double *)(base + o_stats);
  h.a = a_nodal;
  h.ctl = (Ctl *)(base + o_ctl);
  h.info = (DevInfo *)(base + o_info);
  h.part = (double *)(base + o_part);
  h.lz = (double *)(base + o_lz);
  h.Tq = (double2 *)(base + o_v[0]);
  h.Tv[0] = (double2 *)(base + o_v[1]);
  h.Tv[1] = (double2 *)(base + o_v[2]);
  h.Z[0] = (double2 *)(base + o_v[3]);
  h.Z[1] = (double2 *)(base + o_v[4]);
  h.W[0] = (double2 *)(base + o_v[5]);
  h.W[1] = (double2 *)(base + o_v[6]);
  h.T = base + o_t;
  int mo = 0;
  for (int ax = 0; ax < 3; ++ax) {
    h.mu[ax] = (const double *)(base + o_mu) + mo;
    h.mu_f[ax] = (const float *)(base + o_muf) + mo;
    h.gemm[ax] = 0;
    h.Wm[ax] = nullptr;
    h.Wmf[ax] = nullptr;
    mo += h.n[ax];
  }
  // coefficient statistics (sum, face bounds, invalid samples), read back
  HIPCHK(wg256::launch_write_desc(h, d_desc, s));
  HIPCHK(wg256::launch_coef_stats(d_desc, h.d, h.M, (double *)(base + o_spart), stats_nblk, stats,
                                  s));
  double st4[4];
  HIPCHK(hipMemcpyAsync(st4, stats, sizeof(st4), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (st4[3] != 0.0) return fail(CSL_ERR_ARG, "coefficient samples must be finite and positive");
  double abar = 0.0;
  if (o.abar_rule == CSL_ABAR_MEAN) abar = st4[0] / (double)h.M;
  else if (o.abar_rule == CSL_ABAR_GEOMEAN) abar = std::sqrt(st4[1] * st4[2]);
  else abar = o.abar;
  h.abar = abar;
  h.abar_f = (float)abar;
  if (beta == 0.0) {
    std::vector<double> mu(nmu);
    int k0 = 0;
    for (int ax = 0; ax < 3; ++ax) {
      const int n = h.n[ax];
      for (int k = 1; k <= n; ++k) {
        const double sv = std::sin((double)k * M_PI / (2.0 * (n + 1)));
        mu[k0 + k - 1] = ax < h.d ? 4.0 * h.h2[ax] * sv * sv : 0.0;
      }
      k0 += n;
    }
    if (preconditioner_singular(h, mu, abar, alpha, beta))
      return fail(CSL_ERR_SINGULAR, "preconditioner is singular: beta = 0 and "
                                    "abar*mu + alpha = 0 for some mode");
  }
  // schedule of a problem's own solve: the 512-thread solver (the FFT runs
  // on every axis), about one tile per workgroup and phase
  const int wg = 512;
  int bpc = 0;
  HIPCHK(solve_occupancy_wg(wg, h.d == 2, false, false, smem, &bpc));
  const int cap = std::max(1, bpc) * sd.cus;
  set_tile_points(h, (int)std::min<long long>(1 << 30, h.M / cap));
  int mt = 1;
  for (int k = 0; k < K_NKINDS; ++k) mt = std::max(mt, h.ntile[k]);
  HIPCHK(wg256::launch_write_desc(h, d_desc, s));
  const SolveParams P = make_params(so.tol, so.maxit, so.check_true_residual, so.timeout_ms,
                                    sd.wall_khz);
  HIPCHK(wg256::launch_init(d_desc, 1, glob, s));
  IOPtr io0{(const double2 *)f, (double2 *)z};
  HIPCHK(solve_launch(wg, h.d == 2, false, false, d_desc, nullptr, io0, 1, P, glob, std::max(1, std::min(mt, cap)),
                      smem, s));
  if (!info) return CSL_OK;
  DevInfo di;
  HIPCHK(hipMemcpyAsync(&di, h.info, sizeof(di), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const csl_status st = info_from_device(di, info);
  if (st != CSL_OK) g_err = std::string("solve ended with status: ") + status_name(st);
  return st;
}

csl_status problem_set_schedule(csl_problem p, int tile_points, int lds_bytes, int block_threads,
                                int tile_elems, hipStream_t s) {
  if (!p) return fail(CSL_ERR_ARG, "problem is NULL");
  if (tile_points < 0) return fail(CSL_ERR_ARG, "tile_points must be >= 0");
  if (tile_elems < 0) return fail(CSL_ERR_ARG, "tile_elems must be >= 0");
  if (lds_bytes != 0 && lds_bytes != 32768 && lds_bytes != 65536)
    return fail(CSL_ERR_ARG, "lds_bytes must be 0, 32768 or 65536");
  if (!valid_block_threads(block_threads))
    return fail(CSL_ERR_ARG, "block_threads must be 0, 256, 512 or 1024");
  if (block_threads == 512 && !p->wg512_ok)
    return fail(CSL_ERR_ARG, "block_threads 512 needs the FFT engine on every axis");
  const int te0 = p->single_te;
  p->single_te = tile_elems;
  const csl_status st = configure_single(p, tile_points, lds_bytes, block_threads, s);
  if (st != CSL_OK) p->single_te = te0;   // the previous schedule stays in force
  return st;
}

csl_status problem_schedule(csl_problem p, csl_batch_tuning *out) {
  if (!p || !out) return fail(CSL_ERR_ARG, "NULL argument");
  *out = csl_batch_tuning{};
  out->tile_points = p->tile_points;
  out->lds_bytes = p->lds_bytes;
  out->grid_size = p->grid1;
  out->block_threads = p->block_threads;
  out->tile_elems = p->single_te;
  return CSL_OK;
}

csl_status problem_tune(csl_problem p, const double *f, double *z, csl_batch_tuning *out,
                        hipStream_t s) {
  if (!p || !f || !z) return fail(CSL_ERR_ARG, "NULL argument");
  if (f == z) return fail(CSL_ERR_ARG, "problem_tune: f and z must not alias");
  const int tp0 = p->tile_points, lds0 = p->lds_bytes, wg0 = p->block_threads,
            te0 = p->single_te;
  // engine sets: the creation-time one and, where the engines were chosen
  // automatically, the FFT on every axis that has one: the creation-time
  // timing runs the default schedule, under which a matrix-core axis can
  // win and then lose once both are tuned
  int mask0 = 0, req = 0;
  for (int ax = 0; ax < p->h.d; ++ax) {
    if (p->h0.gemm[ax]) mask0 |= 1 << ax;
    if (gemm_required(p->h.n[ax])) req |= 1 << ax;
  }
  const int nmask = (p->opts.dst_engine == CSL_DST_AUTO && mask0 != req) ? 2 : 1;
  const int masks[2] = {mask0, req};
  const int gcode = p->opts.dst_engine == CSL_DST_GEMM16 ? 2 : 1;
  auto set_mask = [&](int m) {
    for (int ax = 0; ax < 3; ++ax) p->h0.gemm[ax] = p->h.gemm[ax] = ((m >> ax) & 1) ? gcode : 0;
    p->wg512_ok = fft_everywhere(p->h0);
  };
  struct Cand {
    int tp, lds, wg, te, mask;
  };
  std::vector<Cand> cands;
  cands.push_back({tp0, lds0, wg0, te0, mask0});
  for (int mi = 0; mi < nmask; ++mi) {
    const int m = masks[mi];
    const bool w512 = fft_everywhere_mask(m);
    const long long per_wg = std::max<long long>(1, p->h.M / std::max(1, p->cap));
    SysDesc hm = p->h0;
    for (int ax = 0; ax < 3; ++ax) hm.gemm[ax] = ((m >> ax) & 1) ? 1 : 0;
    const bool w1024 = plane_ok(hm);
    for (int wg : {256, 512, 1024}) {
      if (wg == 512 && !w512) continue;
      if (wg == 1024 && !w1024) continue;
      for (int lds : {32768, 65536}) {
        if (wg == 1024 && lds != 65536) continue;   // the plane instance's own budget
        std::vector<long long> tps;
        for (long long tp : {0LL, 1LL, per_wg / 2, per_wg * 2, per_wg * 4, per_wg * 8, 4096LL, 8192LL})
          if (tp >= 0 && tp <= (1LL << 30) && std::find(tps.begin(), tps.end(), tp) == tps.end())
            tps.push_back(tp);
        for (long long tp : tps)
          if (!((int)tp == tp0 && lds == lds0 && wg == wg0 && te0 == 0 && m == mask0))
            cands.push_back({(int)tp, lds, wg, 0, m});
      }
      if (p->h.M <= kSmallChunkPoints)
        for (int te : kSmallChunkElems)
          for (long long tp : {0LL, 1LL, per_wg})
            if (!((int)tp == tp0 && wg == wg0 && te == te0 && m == mask0))
              cands.push_back({(int)tp, 32768, wg, te, m});
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(CSL_ERR_HIP, "hipEventCreate failed");
  }
  const SolveParams P = make_params(0.0, 0, 1, 0, p->wall_khz);
  double best = INFINITY, first = INFINITY;
  int best_tp = tp0, best_lds = lds0, best_wg = wg0, best_te = te0, best_mask = mask0, timed = 0;
  csl_status st = CSL_OK;
  for (size_t c = 0; c < cands.size() && st == CSL_OK; ++c) {
    set_mask(cands[c].mask);
    p->single_te = cands[c].te;
    st = configure_single(p, cands[c].tp, cands[c].lds, cands[c].wg, s);
    if (st == CSL_ERR_ARG && cands[c].te > 0) {   // more chunks than partial-sum slots
      st = CSL_OK;
      continue;
    }
    if (st != CSL_OK) break;
    if (c > 0 && p->lds_bytes != cands[c].lds) continue;   // budget not applicable
    st = run_single(p, (const double2 *)f, (double2 *)z, P, s);   // warm-up
    float ms = 0.f, tot = 0.f;
    const int reps = 2;
    for (int r = 0; r < reps && st == CSL_OK; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess) st = fail(CSL_ERR_HIP, "hipEventRecord failed");
      if (st == CSL_OK) st = run_single(p, (const double2 *)f, (double2 *)z, P, s);
      if (st == CSL_OK && (hipEventRecord(e1, s) != hipSuccess ||
                           hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(CSL_ERR_HIP, "event timing failed");
      tot += ms;
    }
    if (st != CSL_OK) break;
    const double avg = tot / reps;
    ++timed;
    if (c == 0) first = avg;
    if (avg < best) {
      best = avg;
      best_tp = cands[c].tp;
      best_lds = p->lds_bytes;
      best_wg = p->block_threads;
      best_te = cands[c].te;
      best_mask = cands[c].mask;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  set_mask(best_mask);
  p->single_te = best_te;
  const csl_status st2 = configure_single(p, best_tp, best_lds, best_wg, s);
  if (st != CSL_OK) return st;
  if (st2 != CSL_OK) return st2;
  if (out) {
    *out = csl_batch_tuning{};
    out->tile_points = best_tp;
    out->lds_bytes = p->lds_bytes;
    out->grid_size = p->grid1;
    out->candidates = timed;
    out->ms = best;
    out->ms_default = first;
    out->block_threads = p->block_threads;
    out->tile_elems = p->single_te;
  }
  return CSL_OK;
}

csl_status minres_adjoint(csl_problem p, const double *z, const double *gz, double *gf,
                          double *galpha, double *gbeta, double *ga, const csl_solve_opts *opts,
                          csl_solve_info *info, hipStream_t s) {
  if (!p || !z || !gz) return fail(CSL_ERR_ARG, "NULL argument");
  if ((const double *)gf == z) return fail(CSL_ERR_ARG, "minres_adjoint: gf and z must not alias");
  csl_solve_opts o{};
  if (opts) o = *opts;
  if (check_solve_opts(o) != CSL_OK) return CSL_ERR_ARG;
  const SolveParams P = make_params(o.tol, o.maxit, o.check_true_residual, o.timeout_ms, p->wall_khz);
  const int M = p->h.M;
  // y = (K + conj(lambda) I)^{-1} G  <=>  A (block) u = conj(G) with u = y;
  // the solve stores conj(u) = conj(y) in ytmp.
  HIPCHK(wg256::launch_conj((const double2 *)gz, p->gtmp, M, s));
  csl_status st = run_single(p, p->gtmp, p->ytmp, P, s);
  if (st != CSL_OK) return st;
  HIPCHK(wg256::launch_adjoint(p->d_desc, p->h.d, M, p->ytmp, (const double2 *)z, (double2 *)gf, ga,
                        p->adj_part, p->adj_nblk, galpha, gbeta, s));
  if (!info) return CSL_OK;
  return fetch_single_info(p, info, s);
}

csl_status batch_create(const csl_problem *problems, int count, const csl_batch_opts *opts,
                        csl_batch *out) {
  if (!out) return fail(CSL_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!problems || count <= 0) return fail(CSL_ERR_ARG, "empty batch");
  csl_batch_opts o{};
  o.use_graph = 1;
  if (opts) o = *opts;
  for (int i = 0; i < count; ++i) {
    if (!problems[i]) return fail(CSL_ERR_ARG, "NULL problem in batch");
    for (int j = 0; j < i; ++j)
      if (problems[j] == problems[i]) return fail(CSL_ERR_ARG, "problem listed twice in batch");
    if (problems[i]->device != problems[0]->device)
      return fail(CSL_ERR_ARG, "batch problems must live on one device");
  }
  csl_batch b = new csl_batch_s();
  b->device = problems[0]->device;
  b->count = count;
  b->probs.assign(problems, problems + count);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o2 = off;
    off += align256(bytes);
    return o2;
  };
  const size_t o_desc = take(sizeof(SysDesc) * count);
  const size_t o_io = take(sizeof(IOPtr) * count);
  const size_t o_io_adj = take(sizeof(IOPtr) * count);
  const size_t o_info = take(sizeof(DevInfo) * count);
  const size_t o_glob = take(sizeof(Glob));
  hipError_t e = hipMalloc(&b->mem, off);
  if (e != hipSuccess) {
    delete b;
    return fail(CSL_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  char *base = (char *)b->mem;
  b->d_desc = (SysDesc *)(base + o_desc);
  b->d_io = (IOPtr *)(base + o_io);
  b->d_io_adj = (IOPtr *)(base + o_io_adj);
  b->d_info = (DevInfo *)(base + o_info);
  b->glob = (Glob *)(base + o_glob);
  auto cleanup = [&](csl_status st, const std::string &msg) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->h_io) (void)hipHostFree(b->h_io);
    if (b->copy_done) (void)hipEventDestroy(b->copy_done);
    (void)hipFree(b->mem);
    delete b;
    return fail(st, msg);
  };
  if (hipHostMalloc((void **)&b->h_io, sizeof(IOPtr) * count, hipHostMallocDefault) != hipSuccess)
    return cleanup(CSL_ERR_HIP, "hipHostMalloc failed");
  if (hipEventCreateWithFlags(&b->copy_done, hipEventDisableTiming) != hipSuccess)
    return cleanup(CSL_ERR_HIP, "hipEventCreate failed");
  if (o.maxit > 16000000) return cleanup(CSL_ERR_ARG, "maxit too large");
  if (!std::isfinite(o.tol)) return cleanup(CSL_ERR_ARG, "tol must be finite");
  if (o.grid_size < 0) return cleanup(CSL_ERR_ARG, "grid_size must be >= 0");
  b->grid_opt = o.grid_size;
  b->params = make_params(o.tol, o.maxit, o.check_true_residual, o.timeout_ms,
                          problems[0]->wall_khz);
  b->use_graph = o.use_graph != 0;
  if (o.lds_bytes != 0 && o.lds_bytes != 32768 && o.lds_bytes != 65536)
    return cleanup(CSL_ERR_ARG, "lds_bytes must be 0, 32768 or 65536");
  if (o.tile_points < 0) return cleanup(CSL_ERR_ARG, "tile_points must be >= 0");
  if (!valid_block_threads(o.block_threads))
    return cleanup(CSL_ERR_ARG, "block_threads must be 0, 256, 512 or 1024");
  b->wg512_ok = true;
  b->all2d = true;
  b->plane_ok = true;
  b->p64 = problems[0]->h0.prec == 0;
  for (int i = 0; i < count; ++i) {
    b->wg512_ok = b->wg512_ok && problems[i]->wg512_ok;
    b->all2d = b->all2d && problems[i]->h.d == 2;
    b->g16 = b->g16 || has_gemm16(problems[i]->h);
    b->plane_ok = b->plane_ok && plane_ok(problems[i]->h0) && (problems[i]->h0.prec == 0) == b->p64;
  }
  if (o.block_threads == 512 && !b->wg512_ok)
    return cleanup(CSL_ERR_ARG, "block_threads 512 needs the FFT engine on every axis of every problem");
  if (o.block_threads == 1024 && !b->plane_ok)
    return cleanup(CSL_ERR_ARG, "block_threads 1024 (the plane phase) needs 3-D problems with one "
                                "preconditioner precision, the FFT on every axis and n0, n1 <= 127 "
                                "(n0 n1 <= 16129 with FP64)");
  {
    // the adjoint solves read conj(G) from each problem's gtmp and write
    // conj(y) to its ytmp
    std::vector<IOPtr> adj(count);
    for (int i = 0; i < count; ++i) adj[i] = IOPtr{problems[i]->gtmp, problems[i]->ytmp};
    if (hipMemcpy(b->d_io_adj, adj.data(), sizeof(IOPtr) * count, hipMemcpyHostToDevice) !=
        hipSuccess)
      return cleanup(CSL_ERR_HIP, "hipMemcpy of the adjoint pointers failed");
  }
  const csl_status st = configure_batch(b, o.tile_points > 0 ? o.tile_points : 8192,
                                        o.lds_bytes, o.block_threads, b->use_graph);
  if (st != CSL_OK) {
    const std::string msg = g_err;
    return cleanup(st, msg);
  }
  *out = b;
  return CSL_OK;
}

csl_status batch_solve(csl_batch b, const double *const *f, double *const *z,
                       csl_solve_info *infos, hipStream_t s) {
  if (!b || !f || !z) return fail(CSL_ERR_ARG, "NULL argument");
  bool same = b->io_valid;
  for (int i = 0; i < b->count; ++i) {
    if (!f[i] || !z[i]) return fail(CSL_ERR_ARG, "NULL vector in batch");
    if (same && (b->h_io[i].f != (const double2 *)f[i] || b->h_io[i].x != (double2 *)z[i]))
      same = false;
  }
  if (!same) {
    // every solution vector is written by its own system while the others
    // read their right-hand sides: no z may be another z or any f
    std::vector<const void *> zs(z, z + b->count);
    std::sort(zs.begin(), zs.end());
    if (std::adjacent_find(zs.begin(), zs.end()) != zs.end())
      return fail(CSL_ERR_ARG, "batch_solve: two systems share a solution vector");
    for (int i = 0; i < b->count; ++i)
      if (std::binary_search(zs.begin(), zs.end(), (const void *)f[i]))
        return fail(CSL_ERR_ARG, "batch_solve: a right-hand side is also a solution vector");
    HIPCHK(hipEventSynchronize(b->copy_done));
    for (int i = 0; i < b->count; ++i) {
      b->h_io[i].f = (const double2 *)f[i];
      b->h_io[i].x = (double2 *)z[i];
    }
    HIPCHK(hipMemcpyAsync(b->d_io, b->h_io, sizeof(IOPtr) * b->count, hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(b->copy_done, s));
    b->io_valid = true;
  }
  if (b->use_graph) {
    HIPCHK(hipGraphLaunch(b->exec, s));
  } else {
    HIPCHK(wg256::launch_init(b->d_desc, b->count, b->glob, s));
    IOPtr none{nullptr, nullptr};
    HIPCHK(solve_launch(b->block_threads, b->all2d, b->g16, b->p64, b->d_desc, b->d_io, none, b->count, b->params,
                        b->glob, b->grid, b->smem, s));
  }
  if (!infos) return CSL_OK;
  std::vector<DevInfo> di(b->count);
  HIPCHK(hipMemcpyAsync(di.data(), b->d_info, sizeof(DevInfo) * b->count, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  csl_status first = CSL_OK;
  int nbad = 0;
  for (int i = 0; i < b->count; ++i) {
    const csl_status st = info_from_device(di[i], &infos[i]);
    if (st != CSL_OK && first == CSL_OK) first = st;
    nbad += st != CSL_OK;
  }
  if (first != CSL_OK)
    g_err = "batch: " + std::to_string(nbad) + " system(s) ended without convergence, the first"
            " with status: " + status_name(first);
  return first;
}

csl_status batch_adjoint(csl_batch b, const double *const *z, const double *const *gz,
                         double *const *gf, double *galpha, double *gbeta, double *ga,
                         const csl_solve_opts *opts, csl_solve_info *infos, hipStream_t s) {
  if (!b || !z || !gz) return fail(CSL_ERR_ARG, "NULL argument");
  for (int i = 0; i < b->count; ++i) {
    if (!z[i] || !gz[i]) return fail(CSL_ERR_ARG, "NULL vector in batch");
    if (gf && gf[i] && (const double *)gf[i] == z[i])
      return fail(CSL_ERR_ARG, "batch_adjoint: gf and z must not alias");
  }
  if (ga) {
    // one coefficient gradient for the whole batch: every system on the
    // grid of the first
    const SysDesc &h0 = b->probs[0]->h;
    for (int i = 1; i < b->count; ++i) {
      const SysDesc &h = b->probs[i]->h;
      bool same = h.d == h0.d;
      for (int ax = 0; ax < 3 && same; ++ax) same = h.n[ax] == h0.n[ax] && h.h2[ax] == h0.h2[ax];
      if (!same)
        return fail(CSL_ERR_ARG, "batch_adjoint: a summed coefficient gradient needs every "
                                 "system on one grid");
    }
  }
  csl_solve_opts o{};
  o.tol = b->params.tol;
  o.maxit = b->params.maxit;
  o.check_true_residual = b->params.check_true;
  if (opts) o = *opts;
  if (check_solve_opts(o) != CSL_OK) return CSL_ERR_ARG;
  const SolveParams P = make_params(o.tol, o.maxit, o.check_true_residual, o.timeout_ms,
                                    b->probs[0]->wall_khz);
  // y_j = (K + conj(lambda_j) I)^{-1} G_j for every system: the block system
  // with right-hand side conj(G_j), all systems in one persistent launch
  for (int i = 0; i < b->count; ++i) {
    const csl_problem p = b->probs[i];
    HIPCHK(wg256::launch_conj((const double2 *)gz[i], p->gtmp, p->h.M, s));
  }
  HIPCHK(wg256::launch_init(b->d_desc, b->count, b->glob, s));
  IOPtr none{nullptr, nullptr};
  HIPCHK(solve_launch(b->block_threads, b->all2d, b->g16, b->p64, b->d_desc, b->d_io_adj, none, b->count, P,
                      b->glob, b->grid, b->smem, s));
  // gradients system by system, in order: ga accumulates the systems'
  // coefficient gradients in a fixed order
  for (int i = 0; i < b->count; ++i) {
    const csl_problem p = b->probs[i];
    HIPCHK(wg256::launch_adjoint(p->d_desc, p->h.d, p->h.M, p->ytmp, (const double2 *)z[i],
                                 gf ? (double2 *)gf[i] : nullptr, ga, p->adj_part, p->adj_nblk,
                                 galpha ? galpha + i : nullptr, gbeta ? gbeta + i : nullptr, s));
  }
  if (!infos) return CSL_OK;
  std::vector<DevInfo> di(b->count);
  HIPCHK(hipMemcpyAsync(di.data(), b->d_info, sizeof(DevInfo) * b->count, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  csl_status first = CSL_OK;
  int nbad = 0;
  for (int i = 0; i < b->count; ++i) {
    const csl_status st = info_from_device(di[i], &infos[i]);
    if (st != CSL_OK && first == CSL_OK) first = st;
    nbad += st != CSL_OK;
  }
  if (first != CSL_OK)
    g_err = "batch adjoint: " + std::to_string(nbad) + " system(s) ended without convergence, "
            "the first with status: " + status_name(first);
  return first;
}

csl_status batch_tune(csl_batch b, const double *const *f, double *const *z,
                      csl_batch_tuning *out, hipStream_t s) {
  if (!b || !f || !z) return fail(CSL_ERR_ARG, "NULL argument");
  const int tp0 = b->tile_points, lds0 = b->lds_bytes, wg0 = b->block_threads;
  // candidates: the creation-time schedule first, then tile sizes around it
  // with both LDS budgets and every allowed workgroup size
  struct Cand {
    int tp, lds, wg;
  };
  std::vector<Cand> cands;
  cands.push_back({tp0, lds0, wg0});
  for (int wg : {256, 512, 1024}) {
    if (wg == 512 && !b->wg512_ok) continue;
    if (wg == 1024 && !b->plane_ok) continue;
    for (int lds : {32768, 65536}) {
      if (wg == 1024 && lds != 65536) continue;   // the plane instance's own budget
      for (int tp : {6144, 8192, 12288, 16384, 24576})
        if (!(tp == tp0 && lds == lds0 && wg == wg0)) cands.push_back({tp, lds, wg});
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(CSL_ERR_HIP, "hipEventCreate failed");
  }
  const bool graph = b->use_graph;
  b->use_graph = false;   // plain launches while timing
  double best = INFINITY, first = INFINITY;
  int best_tp = tp0, best_lds = lds0, best_wg = wg0, timed = 0;
  csl_status st = CSL_OK;
  for (size_t c = 0; c < cands.size() && st == CSL_OK; ++c) {
    st = configure_batch(b, cands[c].tp, cands[c].lds, cands[c].wg, false);
    if (st != CSL_OK) break;
    if (b->lds_bytes != cands[c].lds && c > 0) continue;   // budget not applicable
    st = batch_solve(b, f, z, nullptr, s);   // warm-up (and io upload)
    if (st != CSL_OK) break;
    float ms = 0.f, tot = 0.f;
    const int reps = 2;
    for (int r = 0; r < reps && st == CSL_OK; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess) st = fail(CSL_ERR_HIP, "hipEventRecord failed");
      if (st == CSL_OK) st = batch_solve(b, f, z, nullptr, s);
      if (st == CSL_OK && (hipEventRecord(e1, s) != hipSuccess ||
                           hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(CSL_ERR_HIP, "event timing failed");
      tot += ms;
    }
    if (st != CSL_OK) break;
    const double avg = tot / reps;
    ++timed;
    if (c == 0) first = avg;
    if (avg < best) {
      best = avg;
      best_tp = cands[c].tp;
      best_lds = b->lds_bytes;
      best_wg = b->block_threads;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->use_graph = graph;
  const csl_status st2 = configure_batch(b, best_tp, best_lds, best_wg, graph);
  if (st != CSL_OK) return st;
  if (st2 != CSL_OK) return st2;
  if (out) {
    *out = csl_batch_tuning{};
    out->tile_points = best_tp;
    out->lds_bytes = b->lds_bytes;
    out->grid_size = b->grid;
    out->candidates = timed;
    out->ms = best;
    out->ms_default = first;
    out->block_threads = b->block_threads;
  }
  return CSL_OK;
}

csl_status batch_schedule(csl_batch b, csl_batch_tuning *out) {
  if (!b || !out) return fail(CSL_ERR_ARG, "NULL argument");
  *out = csl_batch_tuning{};
  out->tile_points = b->tile_points;
  out->lds_bytes = b->lds_bytes;
  out->grid_size = b->grid;
  out->block_threads = b->block_threads;
  return CSL_OK;
}

static void free_paradiag(csl_paradiag pd) {
  if (!pd) return;
  if (pd->batch) (void)batch_destroy(pd->batch);
  for (csl_problem p : pd->probs) free_problem(p);
  if (pd->mem) (void)hipFree(pd->mem);
  delete pd;
}

csl_status paradiag_create(const csl_grid *grid, const double *a_nodal, int steps, double tau,
                           double alpha_c, const csl_problem_opts *popts,
                           const csl_batch_opts *bopts, hipStream_t s, csl_paradiag *out) {
  if (!out) return fail(CSL_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (steps < 8 || steps > 1024 || (steps & (steps - 1)) != 0)
    return fail(CSL_ERR_ARG, "steps must be a power of two between 8 and 1024");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(CSL_ERR_ARG, "tau must be finite and > 0");
  if (!(alpha_c > 0.0 && alpha_c <= 1.0)) return fail(CSL_ERR_ARG, "alpha_c must be in (0, 1]");
  csl_paradiag pd = new csl_paradiag_s();
  pd->L = steps;
  pd->lg = ilog2(steps);
  pd->tau = tau;
  pd->alpha_c = alpha_c;
  const double r = std::pow(alpha_c, 1.0 / steps);
  for (int j = 0; j < steps; ++j) {
    // D_j = (1 - alpha^(1/L) exp(-2 pi i j / L)) / tau
    const double th = 2.0 * M_PI * j / steps;
    const double re = (1.0 - r * std::cos(th)) / tau, im = r * std::sin(th) / tau;
    pd->dre.push_back(re);
    pd->dim.push_back(im);
    csl_problem p = nullptr;
    const csl_status st = create_problem(grid, a_nodal, re, im, popts, s, &p);
    if (st != CSL_OK) {
      const std::string msg = g_err;
      free_paradiag(pd);
      return fail(st, "paradiag mode " + std::to_string(j) + ": " + msg);
    }
    pd->probs.push_back(p);
  }
  pd->device = pd->probs[0]->device;
  pd->M = pd->probs[0]->h.M;
  const size_t vec = align256(sizeof(double2) * (size_t)pd->M * steps);
  hipError_t e = hipMalloc(&pd->mem, 2 * vec);
  if (e != hipSuccess) {
    free_paradiag(pd);
    return fail(CSL_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  pd->rt = (double2 *)pd->mem;
  pd->ut = (double2 *)((char *)pd->mem + vec);
  for (int j = 0; j < steps; ++j) {
    pd->fptr.push_back((const double *)(pd->rt + (size_t)j * pd->M));
    pd->zptr.push_back((double *)(pd->ut + (size_t)j * pd->M));
  }
  const csl_status st = batch_create(pd->probs.data(), steps, bopts, &pd->batch);
  if (st != CSL_OK) {
    const std::string msg = g_err;
    free_paradiag(pd);
    return fail(st, msg);
  }
  *out = pd;
  return CSL_OK;
}

csl_status paradiag_shift(csl_paradiag pd, int j, double *alpha, double *beta) {
  if (!pd || !alpha || !beta) return fail(CSL_ERR_ARG, "NULL argument");
  if (j < 0 || j >= pd->L) return fail(CSL_ERR_ARG, "mode index out of range");
  *alpha = pd->dre[j];
  *beta = pd->dim[j];
  return CSL_OK;
}

csl_status paradiag_transform(csl_paradiag pd, const double *x, double *y, int inverse,
                              hipStream_t s) {
  if (!pd || !x || !y) return fail(CSL_ERR_ARG, "NULL argument");
  if (x == y) return fail(CSL_ERR_ARG, "paradiag_transform: x and y must not alias");
  HIPCHK(wg256::launch_step_transform((const double2 *)x, (double2 *)y, pd->M, pd->lg,
                                      pd->alpha_c, inverse ? 1 : 0, s));
  return CSL_OK;
}

csl_status paradiag_solve(csl_paradiag pd, const double *r, double *u, csl_solve_info *infos,
                          hipStream_t s) {
  if (!pd || !r || !u) return fail(CSL_ERR_ARG, "NULL argument");
  if (r == u) return fail(CSL_ERR_ARG, "paradiag_solve: r and u must not alias");
  HIPCHK(wg256::launch_step_transform((const double2 *)r, pd->rt, pd->M, pd->lg, pd->alpha_c, 0, s));
  const csl_status st = batch_solve(pd->batch, pd->fptr.data(), pd->zptr.data(), infos, s);
  if (st != CSL_OK && st != CSL_ERR_NOT_CONVERGED && st != CSL_ERR_BREAKDOWN &&
      st != CSL_ERR_NONFINITE && st != CSL_ERR_TIMEOUT)
    return st;
  const std::string msg = g_err;
  HIPCHK(wg256::launch_step_transform(pd->ut, (double2 *)u, pd->M, pd->lg, pd->alpha_c, 1, s));
  if (st != CSL_OK) g_err = msg;
  return st;
}

csl_status paradiag_tune(csl_paradiag pd, const double *r, csl_batch_tuning *out, hipStream_t s) {
  if (!pd || !r) return fail(CSL_ERR_ARG, "NULL argument");
  HIPCHK(wg256::launch_step_transform((const double2 *)r, pd->rt, pd->M, pd->lg, pd->alpha_c, 0, s));
  return batch_tune(pd->batch, pd->fptr.data(), pd->zptr.data(), out, s);
}

csl_status paradiag_batch(csl_paradiag pd, csl_batch *out) {
  if (!pd || !out) return fail(CSL_ERR_ARG, "NULL argument");
  *out = pd->batch;
  return CSL_OK;
}

csl_status paradiag_destroy(csl_paradiag pd) {
  if (!pd) return fail(CSL_ERR_ARG, "paradiag is NULL");
  free_paradiag(pd);
  return CSL_OK;
}

csl_status batch_destroy(csl_batch b) {
  if (!b) return fail(CSL_ERR_ARG, "batch is NULL");
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->copy_done) (void)hipEventDestroy(b->copy_done);
  if (b->h_io) (void)hipHostFree(b->h_io);
  if (b->mem) (void)hipFree(b->mem);
  delete b;
  return CSL_OK;
}

}  // extern "C"
