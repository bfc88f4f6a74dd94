// Structures shared by the host runtime and the gfx950 kernels of the
// absolute-value preconditioned MINRES solver (arXiv:2408.00488).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csl {

constexpr int TWN = 2048;      // twiddle table length = longest FFT
constexpr int MAX_LG = 11;     // log2(TWN)

// Phase kinds of one MINRES iteration.  The Lanczos vectors are kept
// transformed along the contiguous axis (W_c v, W_c the orthonormal sine
// transform of that axis, which is its own inverse); inner products are
// unchanged by it.  A 2-D iteration j is X, Y, Z; a 3-D one X, Y1, Y, Y1I, Z,
// or X, Y, Z with the plane pass (SysDesc::plane).
enum Kind : int {
  K_X = 0,    // contiguous-axis rows: q = A zhat_j (stencil), delta_j partial,
              // forward transform of q -> Tq (FP64).  Iteration 0: W_c f -> Tv_1
  K_Y1 = 1,   // 3-D axis 1 columns: recurrence Tv_{j+1} = Tq - (delta/gamma) Tv_j
              // - (gamma/gamma_old) Tv_{j-1}, forward transform -> T
  K_Y = 2,    // axis 0 columns: forward transform, per-mode factor, inverse.
              // 2-D: also the recurrence on input and <T, Tv_{j+1}> on output
  K_Y1I = 3,  // 3-D axis 1 columns: inverse transform, <T, Tv_{j+1}> partial
  K_Z = 4,    // contiguous-axis rows: inverse transform -> zhat_{j+1}; update
              // w_{j+1} and x_j of step j
  K_PR = 5,   // rows: true residual ||f - A x||^2 partial
  K_NKINDS = 6,
  K_DONE = 15
};

// Ticket word of a system: [iter:24 | owned:1 | kind:7 | next tile:32]; owned
// marks a phase whose first tiles belong to the workgroups of a fully
// resident single-system grid (see the solver's scheduler).
__host__ __device__ inline uint64_t make_word(int iter, int kind) {
  return ((uint64_t)(uint32_t)iter << 40) | ((uint64_t)(uint32_t)kind << 32);
}
constexpr uint64_t kWordOwned = 1ull << 39;
__host__ __device__ inline int word_iter(uint64_t w) { return (int)(w >> 40); }
__host__ __device__ inline int word_kind(uint64_t w) { return (int)((w >> 32) & 0x7f); }
__host__ __device__ inline bool word_owned(uint64_t w) { return (w & kWordOwned) != 0; }
__host__ __device__ inline uint32_t word_next(uint64_t w) { return (uint32_t)w; }

// Per-system control block: scheduling state and MINRES scalars.
struct alignas(64) Ctl {
  unsigned long long word;   // ticket word (atomic)
  unsigned int done;         // tiles of the current phase completed (atomic)
  int finishing;             // -1, or the status to report after a final PR
  int after_z;               // 0: next iteration, 1: residual check, 2: final
  // Lanczos / Givens scalars (FP64, written only by phase epilogues)
  double gamma, gamma_old;   // gamma_j, gamma_{j-1}
  double c, c_old, s, s_old; // rotations c_j, c_{j-1}, s_j, s_{j-1}
  double eta, eta0;          // residual recurrence
  double delta;              // delta_j
  double bnorm;              // ||f||_2
  double e1, e2, e3, ceta;   // update of w and x of the current step
  double e1p, e2p, e3p, cetap;   // the previous step's, while its update is deferred
  int zmode;                 // what the K_Z phase does (ZM_*)
  int pend;                  // 1: the previous step's update is deferred
  int fin_status, fin_iters; // finish after a ZM_FLUSH phase
  int owned_ok;              // every workgroup of the solver's grid has started
};

// K_Z phase modes.  The w/x updates of MINRES run two steps at a time: a
// step whose update is deferred (ZM_DEFER) only writes zhat_{j+1}; the next
// K_Z phase then applies both steps in one pass over w, x and zhat
// (ZM_PAIR), which halves the reads and writes of w and x.  ZM_SINGLE
// applies one step (before a residual check or the end); ZM_FLUSH applies
// a deferred step alone and ends the solve (breakdown, non-finite values).
enum { ZM_DEFER = 0, ZM_SINGLE = 1, ZM_PAIR = 2, ZM_FLUSH = 3 };

// Result record of one system (device side).
struct DevInfo {
  int status;
  int iters;
  double relres_est;
  double relres_true;
};

// Geometry and data of one system, as the kernels see it.
struct SysDesc {
  int d;          // 2 or 3
  int n[3];       // interior points per axis (axis d-1 contiguous)
  int st[3];      // element strides per axis
  int lg[3];      // log2 of the FFT length 2(n+1) per axis
  int M;          // points
  int rows;       // M / n[d-1]: lines along the contiguous axis
  int prec;       // 0 = FP64 preconditioner, 1 = FP32
  int lpt_x;      // rows per tile of the FP64 contiguous-axis pass (K_X)
  int lpt_z;      // rows per tile of the preconditioner-precision row pass
  int lpt_s[2];   // lines per tile of the strided passes along axes 0, 1
  int lgB;        // log2 of the block width B of the column-blocked layout
                  // (= lines per strided tile): Tq, Tv and T store element
                  // (row, c) at ((c / B) rows + row) B + c % B, so a strided
                  // tile's lines are one contiguous block
  int rpt;        // rows per tile of the residual pass
  int plane;      // 3-D: the transforms along axes 1 and 0 in one phase (K_Y), on
                  // the real or the imaginary part of one plane of those axes at
                  // a time held in LDS (lgB = 0; Tq, Tv and T hold all real
                  // parts, then all imaginary parts, each with the plane of
                  // contiguous-axis index c contiguous)
  int nchunk[K_NKINDS];  // LDS-sized chunks of each phase kind
  int cpt[K_NKINDS];     // chunks per tile (one scheduling unit)
  int ntile[K_NKINDS];   // ceil(nchunk / cpt)
  int maxtile;
  double h2[3];   // 1 / h_k^2
  double alpha, beta, abar;
  float alpha_f, beta_f, abar_f;
  const double *a;         // nodal coefficient (face coefficients are formed from it)
  int gemm[3];             // sine transforms along this axis by a matrix product on
                           // the matrix cores: 0 no (FFT), 1 in the preconditioner's
                           // precision, 2 FP16 products of split operands (FP32
                           // preconditioner only; the FP64 row pass keeps 1)
  const double *Wm[3];     // padded orthonormal DST-I matrix per axis (FP64), if gemm
  const float *Wmf[3];     // FP32 copy
  const void *Wmh[3];      // FP16 high and low parts of 2^kGemm16Shift W, if gemm == 2
  const double *mu[3];     // per-axis eigenvalues of L, FP64
  const float *mu_f[3];    // FP32 copies
  double2 *Tq;             // W_c (A zhat_j)               (column-blocked)
  double2 *Tv[2];          // W_c v_m, by parity of m       (column-blocked)
  void *T;                 // preconditioner intermediate (double2 or float2;
                           // column-blocked)
  double2 *Z[2];           // zhat_m = P^{-1} v_m / gamma_m, by parity of m
  double2 *W[2];           // search directions w_m, by parity of m
  double *part;            // per-tile partial sums
  Ctl *ctl;
  DevInfo *info;
  // Lanczos coefficients of the last solve: lz[2 (j - 1)] = delta_j,
  // lz[2 (j - 1) + 1] = gamma_{j+1} for j <= kLanczosCap; lz[2 kLanczosCap]
  // = the number of steps recorded
  double *lz;
};

constexpr int kLanczosCap = 4096;
// Dynamic LDS of the plane-phase solver instances (the whole 160 KiB of a CU
// less a margin for their static variables), and what a plane tile needs of
// it: one part of the plane in the preconditioner precision (eb bytes per
// value, padded to 128 bytes), one line buffer of 256 complex values per wave
// (nwaves of them), the twiddles of both FFT lengths (one table when they
// are equal; the FFTs have 2 (n + 1) points in FP32, n + 1 in FP64).
constexpr int kPlaneLdsBytes = 163840 - 512;
__host__ __device__ inline int plane_lds_bytes(int n0, int n1, int lg0, int lg1, int eb, int nwaves) {
  const int pb = (n0 * n1 * eb + 127) & ~127;
  const int h = eb == 8 ? 1 : 0;
  const int t0 = (1 << (lg0 - h)) / 4, t1 = (1 << (lg1 - h)) / 4;
  const int ntw = lg0 == lg1 ? t0 : t0 + t1;
  return pb + nwaves * 256 * 2 * eb + ntw * 2 * eb;
}
// The FP16 split-product engine stores the sine matrix scaled by 2^8, so that
// the low parts of its entries stay normal FP16 numbers.
constexpr int kGemm16Shift = 8;

// Right-hand side and output of one system for one solve.
struct IOPtr {
  const double2 *f;
  double2 *x;   // user solution z (stored as conj of the block iterate)
};

// Parameters of one solve launch (shared by every system of a batch).
struct SolveParams {
  double tol;
  int maxit;
  int check_true;
  long long timeout_ticks;   // wall-clock ticks before idle workgroups abort
};

// Launch-wide state of a persistent solve.
struct Glob {
  int active;          // systems not finished
  int error;           // nonzero: abort (time limit)
  int arrived;         // workgroups of the solver's grid that have started
  int pad[13];
};

}  // namespace csl
