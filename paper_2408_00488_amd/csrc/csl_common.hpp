// Structures shared by the host runtime and the gfx950 kernels of the
// absolute-value preconditioned MINRES solver (arXiv:2408.00488).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csl {

constexpr int NT = 256;        // threads per workgroup (4 wave64)
constexpr int TWN = 2048;      // twiddle table length = longest FFT
constexpr int MAX_LG = 11;     // log2(TWN)

// Phase kinds of one MINRES iteration (the order of a 3-D iteration is
// RF, F1, MID, I1, RI, PA [, PR]; a 2-D one skips F1 and I1).
enum Kind : int {
  K_RF = 0,   // sine transform along the contiguous axis; source = new
              // Lanczos vector (stencil + three-term recurrence) or f
  K_F1 = 1,   // 3-D: forward sine transform along axis 1
  K_MID = 2,  // axis 0: forward transform, per-mode scaling, inverse
  K_I1 = 3,   // 3-D: inverse transform along axis 1
  K_RI = 4,   // inverse transform along the contiguous axis -> z, <z, v>
  K_PA = 5,   // w/x update of the previous step + delta = <z, A z>
  K_PR = 6,   // true residual ||f - A x||^2
  K_NKINDS = 7,
  K_DONE = 15
};

// Ticket word of a system: [iter:24 | kind:8 | next tile:32].
__host__ __device__ inline uint64_t make_word(int iter, int kind) {
  return ((uint64_t)(uint32_t)iter << 40) | ((uint64_t)(uint32_t)kind << 32);
}
__host__ __device__ inline int word_iter(uint64_t w) { return (int)(w >> 40); }
__host__ __device__ inline int word_kind(uint64_t w) { return (int)((w >> 32) & 0xff); }
__host__ __device__ inline uint32_t word_next(uint64_t w) { return (uint32_t)w; }

// Per-system control block: scheduling state and MINRES scalars.
struct alignas(64) Ctl {
  unsigned long long word;   // ticket word (atomic)
  unsigned int done;         // tiles of the current phase completed (atomic)
  int finishing;             // -1, or the status to report after a final PR
  // Lanczos / Givens scalars (FP64, written only by phase epilogues)
  double gamma, gamma_old;   // gamma_j, gamma_{j-1}
  double c, c_old, s, s_old; // rotations c_j, c_{j-1}, s_j, s_{j-1}
  double eta, eta0;          // residual recurrence
  double delta;              // delta_j
  double bnorm;              // ||f||_2
  double e1, e2, e3, ceta;   // pending update of w and x
  int has_update;
  int pad;
};

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
  int lpt[3];     // lines per tile of the sine-transform pass along each axis
  int rpt;        // rows per tile of the pointwise passes
  int ntile[K_NKINDS];
  int maxtile;
  double h2[3];   // 1 / h_k^2
  double alpha, beta, abar;
  float alpha_f, beta_f, abar_f;
  const double *a;         // nodal coefficient
  const double *mu[3];     // per-axis eigenvalues of L, FP64
  const float *mu_f[3];    // FP32 copies
  double2 *V[2];           // Lanczos vectors v (by parity of the index)
  double2 *Z[2];           // preconditioned vectors z
  double2 *W[2];           // search directions w
  void *T;                 // sine-transform intermediate (double2 or float2)
  double *part;            // per-tile partial sums
  Ctl *ctl;
  DevInfo *info;
  // solve parameters
  double tol;
  int maxit;
  int check_true;
};

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
  int pad[14];
};

}  // namespace csl
