// gfx950 kernels of the absolute-value preconditioned MINRES solver
// (arXiv:2408.00488): the persistent multi-system scheduler, the phase tiles
// of one MINRES iteration, stand-alone A and P^{-1} applications, the
// adjoint reduction and the coefficient set-up reductions.
#include <math.h>

#include "csl_device.hpp"
#include "csl_kernels.hpp"

namespace csl {

template <typename R>
__device__ __forceinline__ Cx<R> to_cx(double2 v) {
  return Cx<R>{(R)v.x, (R)v.y};
}

// ---------------------------------------------------------------------------
// One tile of a sine-transform pass.
//   MINRES mode (STANDALONE = false):
//     K_RF  iter 0: source f (also ||f||^2 partial, zero the output x)
//     K_RF  iter j: source v_{j+1} = A zhat_j - (delta_j/gamma_j) v_j
//                   - (gamma_j/gamma_{j-1}) v_{j-1}, written to V[(j+1)&1]
//     K_F1, K_MID, K_I1: T -> T
//     K_RI  iter j: T -> z_{j+1} in Z[(j+1)&1] and the partial <z_{j+1}, v_{j+1}>
//   Stand-alone P^{-1} (STANDALONE = true): first pass reads x, last writes y.
// The transform of every pass is the orthonormal DST-I (its own inverse);
// K_MID applies forward transform, per-mode factor, inverse transform.
// ---------------------------------------------------------------------------
template <typename R, int D, bool STANDALONE>
__device__ void tile_line(const SysDesc &S, const IOPtr &io, int kind, int iter, int tile,
                          char *smem, double *red) {
  Cx<R> *buf = reinterpret_cast<Cx<R> *>(smem);
  const int ax = (kind == K_RF || kind == K_RI) ? D - 1 : (kind == K_MID ? 0 : 1);
  const LineTile t = line_tile(S, ax, tile);
  Cx<R> *T = reinterpret_cast<Cx<R> *>(S.T);
  double acc = 0.0;

  // ---------------- fill
  if (kind == K_RF && STANDALONE) {
    const double2 *__restrict__ x = io.f;
    lines_fill<R>(buf, t, [&](int, int, int p) { return to_cx<R>(x[p]); });
  } else if (kind == K_RF && iter == 0) {
    const double2 *__restrict__ f = io.f;
    double2 *__restrict__ X = io.x;
    lines_fill<R>(buf, t, [&](int, int, int p) {
      const double2 v = f[p];
      acc += v.x * v.x + v.y * v.y;
      X[p] = make_double2(0.0, 0.0);
      return to_cx<R>(v);
    });
  } else if (kind == K_RF) {
    const int j = iter;
    const Ctl *C = S.ctl;
    const double g = ld_ctl(&C->gamma), go = ld_ctl(&C->gamma_old);
    const double dl = ld_ctl(&C->delta);
    const double ig = 1.0 / g, cd = dl / g, cg = g / go;
    const double al = S.alpha, be = S.beta;
    const double2 *__restrict__ zj = S.Z[j & 1];
    const double2 *__restrict__ vj = (j == 1) ? io.f : S.V[j & 1];
    const double2 *__restrict__ vjm1 = (j == 2) ? io.f : S.V[(j - 1) & 1];
    double2 *vout = S.V[(j + 1) & 1];
    const bool has_vm1 = j >= 2;
    const double *__restrict__ a = S.a;
    lines_fill<R>(buf, t, [&](int l, int r, int p) {
      int idx[3];
      row_index<D>(S, t.row0 + l, r, idx);
      const double2 kz = stencil_K<D>(S, a, zj, p, idx);
      const double2 zz = zj[p];
      const double zx = zz.x * ig, zy = zz.y * ig;
      const double kx = kz.x * ig, ky = kz.y * ig;
      // q = A zhat in complex storage = conj(K zhat + conj(lambda) zhat)
      const double qx = kx + al * zx + be * zy;
      const double qy = -(ky + al * zy - be * zx);
      const double2 v1 = vj[p];
      double vx = qx - cd * v1.x, vy = qy - cd * v1.y;
      if (has_vm1) {
        const double2 v0 = vjm1[p];
        vx -= cg * v0.x;
        vy -= cg * v0.y;
      }
      vout[p] = make_double2(vx, vy);
      return Cx<R>{(R)vx, (R)vy};
    });
  } else {
    lines_fill<R>(buf, t, [&](int, int, int p) { return T[p]; });
  }

  fft_lines<R>(buf, t.nl, t.lg);

  if (kind == K_MID) {
    const R ab = (sizeof(R) == 8) ? (R)S.abar : (R)S.abar_f;
    const R al = (sizeof(R) == 8) ? (R)S.alpha : (R)S.alpha_f;
    const R be = (sizeof(R) == 8) ? (R)S.beta : (R)S.beta_f;
    const R *mu0;
    const R *mu1;
    const R *mu2;
    if constexpr (sizeof(R) == 8) {
      mu0 = reinterpret_cast<const R *>(S.mu[0]);
      mu1 = reinterpret_cast<const R *>(S.mu[1]);
      mu2 = reinterpret_cast<const R *>(S.mu[2]);
    } else {
      mu0 = reinterpret_cast<const R *>(S.mu_f[0]);
      mu1 = reinterpret_cast<const R *>(S.mu_f[1]);
      mu2 = reinterpret_cast<const R *>(S.mu_f[2]);
    }
    lines_scale_extend<R>(buf, t, [&](int l, int r) -> R {
      R lam;
      if (D == 2) {
        lam = mu0[r] + mu1[t.c0 + l];
      } else {
        lam = (mu0[r] + mu1[t.outer]) + mu2[t.c0 + l];
      }
      const R sh = ab * lam + al;
      return (R)1 / sqrt(sh * sh + be * be);
    });
    fft_lines<R>(buf, t.nl, t.lg);
  }

  // ---------------- store
  if (kind == K_RI && STANDALONE) {
    double2 *__restrict__ y = io.x;
    lines_store<R>(buf, t, [&](int, int, int p, Cx<R> v) {
      y[p] = make_double2((double)v.x, (double)v.y);
    });
  } else if (kind == K_RI) {
    const int j = iter;
    double2 *__restrict__ zout = S.Z[(j + 1) & 1];
    const double2 *__restrict__ partner = (j == 0) ? io.f : S.V[(j + 1) & 1];
    lines_store<R>(buf, t, [&](int, int, int p, Cx<R> v) {
      const double2 z = make_double2((double)v.x, (double)v.y);
      zout[p] = z;
      const double2 w = partner[p];
      acc += z.x * w.x + z.y * w.y;
    });
  } else {
    lines_store<R>(buf, t, [&](int, int, int p, Cx<R> v) { T[p] = v; });
  }
  if (!STANDALONE && (kind == K_RI || (kind == K_RF && iter == 0))) {
    const double s = wg_sum(acc, red);
    if (threadIdx.x == 0) S.part[tile] = s;
  }
}

// ---------------------------------------------------------------------------
// Pointwise phase PA of iteration j: apply the pending update of step j-1
//   w_j = (zhat_{j-1} - e3 w_{j-2} - e2 w_{j-1}) / e1,  x_{j-1} = x_{j-2} + ceta w_j
// (x held as its conjugate, the user's z), and the partial of
// delta_j = <zhat_j, A zhat_j>.
// ---------------------------------------------------------------------------
template <int D>
__device__ void tile_PA(const SysDesc &S, const IOPtr &io, int j, int tile, double *red) {
  const Ctl *C = S.ctl;
  const int upd = ld_ctl(&C->has_update);
  const double g = ld_ctl(&C->gamma), go = ld_ctl(&C->gamma_old);
  const double e1 = ld_ctl(&C->e1), e2 = ld_ctl(&C->e2), e3 = ld_ctl(&C->e3);
  const double ceta = ld_ctl(&C->ceta);
  const int nlast = S.n[D - 1];
  const int r0 = tile * S.rpt;
  const int r1 = min(S.rows, r0 + S.rpt);
  const int p0 = r0 * nlast, p1 = r1 * nlast;
  const double2 *__restrict__ zj = S.Z[j & 1];
  const double2 *__restrict__ zjm1 = S.Z[(j - 1) & 1];
  double2 *wnew = S.W[j & 1];
  const double2 *__restrict__ wjm1 = S.W[(j - 1) & 1];
  double2 *__restrict__ X = io.x;
  const bool use_wm2 = j > 3, use_wm1 = j > 2, use_x = j > 2;
  const bool do_delta = (g != 0.0);
  const double igo = 1.0 / go;
  const double ig = do_delta ? 1.0 / g : 0.0;
  const double al = S.alpha, be = S.beta;
  const double *__restrict__ a = S.a;
  double acc = 0.0;
  for (int p = p0 + (int)threadIdx.x; p < p1; p += NT) {
    if (upd) {
      const double2 zz = zjm1[p];
      double wx = zz.x * igo, wy = zz.y * igo;
      if (use_wm2) {
        const double2 w0 = wnew[p];
        wx -= e3 * w0.x;
        wy -= e3 * w0.y;
      }
      if (use_wm1) {
        const double2 w1 = wjm1[p];
        wx -= e2 * w1.x;
        wy -= e2 * w1.y;
      }
      wx /= e1;
      wy /= e1;
      wnew[p] = make_double2(wx, wy);
      double2 xv = use_x ? X[p] : make_double2(0.0, 0.0);
      xv.x += ceta * wx;
      xv.y -= ceta * wy;
      X[p] = xv;
    }
    if (do_delta) {
      const int row = p / nlast;
      int idx[3];
      row_index<D>(S, row, p - row * nlast, idx);
      const double2 kz = stencil_K<D>(S, a, zj, p, idx);
      const double2 zz = zj[p];
      const double zx = zz.x * ig, zy = zz.y * ig;
      const double kx = kz.x * ig, ky = kz.y * ig;
      const double qx = kx + al * zx + be * zy;
      const double qy = -(ky + al * zy - be * zx);
      acc += zx * qx + zy * qy;
    }
  }
  const double s = wg_sum(acc, red);
  if (threadIdx.x == 0) S.part[tile] = s;
}

// True residual partial ||f - (K + lambda I) z||^2 with z the user output.
template <int D>
__device__ void tile_PR(const SysDesc &S, const IOPtr &io, int tile, double *red) {
  const int nlast = S.n[D - 1];
  const int r0 = tile * S.rpt;
  const int r1 = min(S.rows, r0 + S.rpt);
  const int p0 = r0 * nlast, p1 = r1 * nlast;
  const double2 *__restrict__ X = io.x;
  const double2 *__restrict__ f = io.f;
  const double al = S.alpha, be = S.beta;
  double acc = 0.0;
  for (int p = p0 + (int)threadIdx.x; p < p1; p += NT) {
    const int row = p / nlast;
    int idx[3];
    row_index<D>(S, row, p - row * nlast, idx);
    const double2 kx = stencil_K<D>(S, S.a, X, p, idx);
    const double2 xv = X[p];
    const double ux = kx.x + al * xv.x - be * xv.y;
    const double uy = kx.y + al * xv.y + be * xv.x;
    const double2 fv = f[p];
    const double rx = fv.x - ux, ry = fv.y - uy;
    acc += rx * rx + ry * ry;
  }
  const double s = wg_sum(acc, red);
  if (threadIdx.x == 0) S.part[tile] = s;
}

__device__ void process_tile(const SysDesc &S, const IOPtr &io, int kind, int iter, int tile,
                             char *smem, double *red) {
  if (kind == K_PA) {
    if (S.d == 3) tile_PA<3>(S, io, iter, tile, red);
    else tile_PA<2>(S, io, iter, tile, red);
  } else if (kind == K_PR) {
    if (S.d == 3) tile_PR<3>(S, io, tile, red);
    else tile_PR<2>(S, io, tile, red);
  } else if (S.prec) {
    if (S.d == 3) tile_line<float, 3, false>(S, io, kind, iter, tile, smem, red);
    else tile_line<float, 2, false>(S, io, kind, iter, tile, smem, red);
  } else {
    if (S.d == 3) tile_line<double, 3, false>(S, io, kind, iter, tile, smem, red);
    else tile_line<double, 2, false>(S, io, kind, iter, tile, smem, red);
  }
}

// ---------------------------------------------------------------------------
// Phase epilogue, run by the workgroup that completed the last tile of a
// phase: sums the tile partials in a fixed order, advances the Lanczos /
// Givens recurrences, takes the stopping decision and publishes the next
// phase of this system.
// ---------------------------------------------------------------------------
__device__ void publish(Ctl *C, int iter, int kind) {
  __hip_atomic_store(&C->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __threadfence();
  __hip_atomic_exchange(&C->word, (unsigned long long)make_word(iter, kind), __ATOMIC_RELEASE,
                        __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void finish(const SysDesc &S, Glob *G, int iter, int status, int iters, double rt) {
  DevInfo *I = S.info;
  I->status = status;
  I->iters = iters;
  I->relres_true = rt;
  __threadfence();
  __hip_atomic_exchange(&S.ctl->word, (unsigned long long)make_word(iter, K_DONE),
                        __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_fetch_add(&G->active, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

enum { ST_OK = 0, ST_NOT_CONVERGED = 3, ST_BREAKDOWN = 4, ST_NONFINITE = 5 };

__device__ void epilogue(const SysDesc &S, const SolveParams &P, int kind, int iter, Glob *G,
                         double *red) {
  const int nt = S.ntile[kind];
  double a = 0.0;
  const bool need_sum = (kind == K_RI || kind == K_PA || kind == K_PR || (kind == K_RF && iter == 0));
  if (need_sum) {
    for (int i = threadIdx.x; i < nt; i += NT) a += S.part[i];
  }
  const double sum = need_sum ? wg_sum(a, red) : 0.0;
  if (threadIdx.x != 0) return;
  Ctl *C = S.ctl;
  const int first_mid = (S.d == 3) ? K_F1 : K_MID;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  switch (kind) {
    case K_RF:
      if (iter == 0) {
        const double bn = sqrt(sum);
        C->bnorm = bn;
        if (!isfinite(bn)) {
          S.info->relres_est = nan;
          finish(S, G, iter, ST_NONFINITE, 0, nan);
        } else if (bn == 0.0) {
          S.info->relres_est = 0.0;
          finish(S, G, iter, ST_OK, 0, 0.0);
        } else {
          publish(C, iter, first_mid);
        }
      } else {
        publish(C, iter, first_mid);
      }
      break;
    case K_F1:
      publish(C, iter, K_MID);
      break;
    case K_MID:
      publish(C, iter, S.d == 3 ? K_I1 : K_RI);
      break;
    case K_I1:
      publish(C, iter, K_RI);
      break;
    case K_RI: {
      const double g2 = sum;
      const int done_iters = iter > 0 ? iter - 1 : 0;
      if (!isfinite(g2)) {
        S.info->relres_est = nan;
        finish(S, G, iter, ST_NONFINITE, done_iters, nan);
        break;
      }
      if (iter == 0) {
        if (g2 <= 0.0) {
          S.info->relres_est = nan;
          finish(S, G, iter, ST_BREAKDOWN, 0, nan);
          break;
        }
        const double g = sqrt(g2);
        C->gamma = g;
        C->gamma_old = 1.0;
        C->eta = g;
        C->eta0 = g;
        C->c = 1.0;
        C->c_old = 1.0;
        C->s = 0.0;
        C->s_old = 0.0;
        C->has_update = 0;
        publish(C, 1, K_PA);
      } else {
        if (g2 < 0.0) {
          finish(S, G, iter, ST_BREAKDOWN, done_iters, nan);
          break;
        }
        const double gn = sqrt(g2);
        const double dl = C->delta, g = C->gamma;
        const double c = C->c, co = C->c_old, s = C->s, so = C->s_old, eta = C->eta;
        const double e0 = c * dl - co * s * g;
        const double e1 = hypot(e0, gn);
        const double e2 = s * dl + co * c * g;
        const double e3 = so * g;
        const double cn = e0 / e1, sn = gn / e1;
        C->e1 = e1;
        C->e2 = e2;
        C->e3 = e3;
        C->ceta = cn * eta;
        C->eta = -sn * eta;
        C->has_update = 1;
        C->c_old = c;
        C->c = cn;
        C->s_old = s;
        C->s = sn;
        C->gamma_old = g;
        C->gamma = gn;
        publish(C, iter + 1, K_PA);
      }
      break;
    }
    case K_PA: {
      C->delta = sum;
      if (!C->has_update) {
        publish(C, iter, K_RF);
        break;
      }
      const int k = iter - 1;
      const double est = fabs(C->eta) / C->eta0;
      S.info->relres_est = est;
      const bool lucky = (C->gamma == 0.0);
      if (!lucky && !isfinite(sum)) {
        finish(S, G, iter, ST_NONFINITE, k, nan);
      } else if (lucky) {
        C->finishing = ST_OK;
        publish(C, iter, K_PR);
      } else if (est <= P.tol) {
        C->finishing = P.check_true ? -1 : ST_OK;
        publish(C, iter, K_PR);
      } else if (k >= P.maxit) {
        C->finishing = ST_NOT_CONVERGED;
        publish(C, iter, K_PR);
      } else {
        publish(C, iter, K_RF);
      }
      break;
    }
    case K_PR: {
      const int k = iter - 1;
      const double rt = sqrt(sum) / C->bnorm;
      if (C->finishing >= 0) {
        finish(S, G, iter, C->finishing, k, rt);
      } else if (rt <= P.tol) {
        finish(S, G, iter, ST_OK, k, rt);
      } else if (k >= P.maxit) {
        finish(S, G, iter, ST_NOT_CONVERGED, k, rt);
      } else {
        publish(C, iter, K_RF);
      }
      break;
    }
    default:
      break;
  }
}

// ---------------------------------------------------------------------------
// Persistent solver: every workgroup repeatedly claims a tile of whichever
// system has one ready, processes it, and the workgroup that completes a
// phase runs its epilogue.  A workgroup never waits while holding a tile,
// so progress does not depend on which workgroups are resident.  Idle
// workgroups exit when every system is done or the time limit passes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void solve_kernel(const SysDesc *__restrict__ sys,
                                                   const IOPtr *__restrict__ io, IOPtr io0,
                                                   int nsys, SolveParams P, Glob *G) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[NT];
  __shared__ int sh_s, sh_tile, sh_kind, sh_iter, sh_last;
  const int tid = threadIdx.x;
  int cur = blockIdx.x % nsys;
  const long long t0 = wall_clock64();
  for (;;) {
    if (tid == 0) {
      int found = -1;
      if (__hip_atomic_load(&G->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0 ||
          __hip_atomic_load(&G->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        found = -2;
      } else {
        for (int k = 0; k < nsys && found == -1; ++k) {
          int s = cur + k;
          if (s >= nsys) s -= nsys;
          Ctl *C = sys[s].ctl;
          const uint64_t w = __hip_atomic_load(&C->word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const int kd = word_kind(w);
          if (kd >= K_NKINDS || word_next(w) >= (uint32_t)sys[s].ntile[kd]) continue;
          const uint64_t w2 = __hip_atomic_fetch_add(&C->word, 1ull, __ATOMIC_ACQUIRE,
                                                     __HIP_MEMORY_SCOPE_AGENT);
          const int kd2 = word_kind(w2);
          if (kd2 < K_NKINDS && word_next(w2) < (uint32_t)sys[s].ntile[kd2]) {
            found = s;
            sh_tile = (int)word_next(w2);
            sh_kind = kd2;
            sh_iter = word_iter(w2);
            cur = s;
          }
        }
        if (found == -1) {
          __builtin_amdgcn_s_sleep(2);
          if (wall_clock64() - t0 > P.timeout_ticks) {
            __hip_atomic_fetch_or(&G->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            found = -2;
          }
        }
      }
      sh_s = found;
    }
    __syncthreads();
    const int s = sh_s;
    if (s == -2) break;
    if (s >= 0) {
      const int kind = sh_kind, iter = sh_iter, tile = sh_tile;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const SysDesc &S = sys[s];
      const IOPtr iop = io ? io[s] : io0;
      process_tile(S, iop, kind, iter, tile, smem, red);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (tid == 0) {
        const unsigned old = __hip_atomic_fetch_add(&S.ctl->done, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        sh_last = (old + 1 == (unsigned)S.ntile[kind]);
      }
      __syncthreads();
      if (sh_last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        epilogue(S, P, kind, iter, G, red);
      }
    }
    __syncthreads();
  }
}

__global__ void init_kernel(const SysDesc *__restrict__ sys, int nsys, Glob *G) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    Ctl *C = sys[s].ctl;
    C->word = make_word(0, K_RF);
    C->done = 0;
    C->finishing = -1;
    C->has_update = 0;
    DevInfo *I = sys[s].info;
    I->status = -1;
    I->iters = 0;
    I->relres_est = 0.0;
    I->relres_true = 0.0;
  }
  if (threadIdx.x == 0) {
    G->active = nsys;
    G->error = 0;
  }
}

// ---------------------------------------------------------------------------
// Stand-alone operators.
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(NT) void apply_A_kernel(const SysDesc *__restrict__ sys,
                                                     const double2 *__restrict__ x,
                                                     double2 *__restrict__ y) {
  const SysDesc &S = *sys;
  const int nlast = S.n[D - 1];
  for (int p = blockIdx.x * NT + threadIdx.x; p < S.M; p += gridDim.x * NT) {
    const int row = p / nlast;
    int idx[3];
    row_index<D>(S, row, p - row * nlast, idx);
    const double2 kx = stencil_K<D>(S, S.a, x, p, idx);
    const double2 xv = x[p];
    // y = (K + lambda I) conj(x) = conj(K x + conj(lambda) x)
    const double ux = kx.x + S.alpha * xv.x + S.beta * xv.y;
    const double uy = kx.y + S.alpha * xv.y - S.beta * xv.x;
    y[p] = make_double2(ux, -uy);
  }
}

template <typename R, int D>
__global__ __launch_bounds__(NT) void pinv_pass_kernel(const SysDesc *__restrict__ sys, int kind,
                                                       const double2 *x, double2 *y) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[NT];
  IOPtr io{x, y};
  tile_line<R, D, true>(*sys, io, kind, 0, blockIdx.x, smem, red);
}

// ---------------------------------------------------------------------------
// Adjoint reduction.  ytil is the adjoint solve's output buffer, which holds
// conj(y); y = (K + conj(lambda) I)^{-1} G.  Per node p:
//   gf_p = y_p,  ga_p += sum_faces dL/dc_e * dc_e/da_p,
// and per-block partials of Re(y^H z) and Im(y^H z).
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(NT) void adjoint_kernel(const SysDesc *__restrict__ sys,
                                                     const double2 *__restrict__ ytil,
                                                     const double2 *__restrict__ z,
                                                     double2 *__restrict__ gf,
                                                     double *__restrict__ ga,
                                                     double *__restrict__ part) {
  __shared__ double red[NT];
  const SysDesc &S = *sys;
  const int nlast = S.n[D - 1];
  const double *__restrict__ a = S.a;
  double sre = 0.0, sim = 0.0;
  for (int p = blockIdx.x * NT + threadIdx.x; p < S.M; p += gridDim.x * NT) {
    const int row = p / nlast;
    int idx[3];
    row_index<D>(S, row, p - row * nlast, idx);
    const double2 yt = ytil[p];
    const double yx = yt.x, yy = -yt.y;
    const double2 zp = z[p];
    if (gf) gf[p] = make_double2(yx, yy);
    sre += yx * zp.x + yy * zp.y;
    sim += yx * zp.y - yy * zp.x;
    if (ga) {
      const double ap = a[p];
      double g = 0.0;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        const int st = S.st[ax];
        const double h2 = S.h2[ax];
        for (int dir = -1; dir <= 1; dir += 2) {
          const bool inside = dir < 0 ? idx[ax] > 0 : idx[ax] < S.n[ax] - 1;
          if (inside) {
            const int q = p + dir * st;
            const double aq = a[q];
            const double2 ytq = ytil[q];
            const double2 zq = z[q];
            const double dyx = yx - ytq.x, dyy = yy + ytq.y;
            const double dzx = zp.x - zq.x, dzy = zp.y - zq.y;
            const double dLdc = -h2 * (dyx * dzx + dyy * dzy);
            const double sm = ap + aq;
            g += dLdc * 2.0 * aq * aq / (sm * sm);
          } else {
            g += -h2 * (yx * zp.x + yy * zp.y);
          }
        }
      }
      ga[p] += g;
    }
  }
  const double r0 = wg_sum(sre, red);
  const double r1 = wg_sum(sim, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r0;
    part[2 * blockIdx.x + 1] = r1;
  }
}

__global__ __launch_bounds__(NT) void adjoint_final_kernel(const double *__restrict__ part,
                                                           int nblk, double *galpha,
                                                           double *gbeta) {
  __shared__ double red[NT];
  double a0 = 0.0, a1 = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT) {
    a0 += part[2 * i];
    a1 += part[2 * i + 1];
  }
  const double re = wg_sum(a0, red);
  const double im = wg_sum(a1, red);
  if (threadIdx.x == 0) {
    if (galpha) *galpha = -re;
    if (gbeta) *gbeta = im;
  }
}

__global__ __launch_bounds__(NT) void conj_kernel(const double2 *__restrict__ x,
                                                  double2 *__restrict__ y, int M) {
  for (int p = blockIdx.x * NT + threadIdx.x; p < M; p += gridDim.x * NT) {
    const double2 v = x[p];
    y[p] = make_double2(v.x, -v.y);
  }
}

// ---------------------------------------------------------------------------
// Coefficient set-up: sum of the nodal samples, min / max over all face
// coefficients (harmonic means inside, a_p on boundary faces), and a count
// of samples that are not finite and positive.
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(NT) void coef_stats_kernel(const SysDesc *__restrict__ sys,
                                                        double *__restrict__ part) {
  __shared__ double red[NT];
  const SysDesc &S = *sys;
  const int nlast = S.n[D - 1];
  const double *__restrict__ a = S.a;
  double sum = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
  for (int p = blockIdx.x * NT + threadIdx.x; p < S.M; p += gridDim.x * NT) {
    const int row = p / nlast;
    int idx[3];
    row_index<D>(S, row, p - row * nlast, idx);
    const double ap = a[p];
    if (!(ap > 0.0) || !isfinite(ap)) bad += 1.0;
    sum += ap;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
      double c;
      if (idx[ax] > 0) {
        const double aq = a[p - S.st[ax]];
        c = 2.0 * ap * aq / (ap + aq);
      } else {
        c = ap;
      }
      mn = fmin(mn, c);
      mx = fmax(mx, c);
      if (idx[ax] == S.n[ax] - 1) {
        mn = fmin(mn, ap);
        mx = fmax(mx, ap);
      }
    }
  }
  const double s0 = wg_sum(sum, red);
  const double s3 = wg_sum(bad, red);
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double s1 = red[0];
  __syncthreads();
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double s2 = red[0];
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = s0;
    part[4 * blockIdx.x + 1] = s1;
    part[4 * blockIdx.x + 2] = s2;
    part[4 * blockIdx.x + 3] = s3;
  }
}

__global__ __launch_bounds__(NT) void coef_stats_final_kernel(const double *__restrict__ part,
                                                              int nblk, double *out) {
  __shared__ double red[NT];
  double s0 = 0.0, s1 = INFINITY, s2 = -INFINITY, s3 = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT) {
    s0 += part[4 * i];
    s1 = fmin(s1, part[4 * i + 1]);
    s2 = fmax(s2, part[4 * i + 2]);
    s3 += part[4 * i + 3];
  }
  const double t0 = wg_sum(s0, red);
  const double t3 = wg_sum(s3, red);
  red[threadIdx.x] = s1;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double t1 = red[0];
  __syncthreads();
  red[threadIdx.x] = s2;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = t0;
    out[1] = t1;
    out[2] = red[0];
    out[3] = t3;
  }
}

// ---------------------------------------------------------------------------
// Host-side launch wrappers (declared in csl_kernels.hpp).
// ---------------------------------------------------------------------------
hipError_t upload_twiddles(const double2 *tw64, const float2 *tw32) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_tw64), tw64, sizeof(double2) * TWN);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tw32), tw32, sizeof(float2) * TWN);
}

hipError_t launch_init(const SysDesc *dsys, int nsys, Glob *G, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(64), 0, s, dsys, nsys, G);
  return hipGetLastError();
}

hipError_t launch_solve(const SysDesc *dsys, const IOPtr *dio, IOPtr io0, int nsys,
                        const SolveParams &P, Glob *G, int grid, size_t smem, hipStream_t s) {
  hipLaunchKernelGGL(solve_kernel, dim3(grid), dim3(NT), smem, s, dsys, dio, io0, nsys, P, G);
  return hipGetLastError();
}

hipError_t solve_occupancy(size_t smem, int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, solve_kernel, NT, smem);
}

hipError_t launch_apply_A(const SysDesc *dsys, int d, int M, const double2 *x, double2 *y,
                          hipStream_t s) {
  const int grid = (M + NT - 1) / NT < 4096 ? (M + NT - 1) / NT : 4096;
  if (d == 3) hipLaunchKernelGGL(apply_A_kernel<3>, dim3(grid), dim3(NT), 0, s, dsys, x, y);
  else hipLaunchKernelGGL(apply_A_kernel<2>, dim3(grid), dim3(NT), 0, s, dsys, x, y);
  return hipGetLastError();
}

hipError_t launch_pinv_pass(const SysDesc *dsys, int d, int prec, int kind, int ntile, size_t smem,
                            const double2 *x, double2 *y, hipStream_t s) {
  if (prec) {
    if (d == 3)
      hipLaunchKernelGGL((pinv_pass_kernel<float, 3>), dim3(ntile), dim3(NT), smem, s, dsys, kind, x, y);
    else
      hipLaunchKernelGGL((pinv_pass_kernel<float, 2>), dim3(ntile), dim3(NT), smem, s, dsys, kind, x, y);
  } else {
    if (d == 3)
      hipLaunchKernelGGL((pinv_pass_kernel<double, 3>), dim3(ntile), dim3(NT), smem, s, dsys, kind, x, y);
    else
      hipLaunchKernelGGL((pinv_pass_kernel<double, 2>), dim3(ntile), dim3(NT), smem, s, dsys, kind, x, y);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(const SysDesc *dsys, int d, int M, const double2 *ytil,
                          const double2 *z, double2 *gf, double *ga, double *part, int nblk,
                          double *galpha, double *gbeta, hipStream_t s) {
  if (d == 3)
    hipLaunchKernelGGL(adjoint_kernel<3>, dim3(nblk), dim3(NT), 0, s, dsys, ytil, z, gf, ga, part);
  else
    hipLaunchKernelGGL(adjoint_kernel<2>, dim3(nblk), dim3(NT), 0, s, dsys, ytil, z, gf, ga, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adjoint_final_kernel, dim3(1), dim3(NT), 0, s, part, nblk, galpha, gbeta);
  return hipGetLastError();
}

hipError_t launch_conj(const double2 *x, double2 *y, int M, hipStream_t s) {
  const int grid = (M + NT - 1) / NT < 4096 ? (M + NT - 1) / NT : 4096;
  hipLaunchKernelGGL(conj_kernel, dim3(grid), dim3(NT), 0, s, x, y, M);
  return hipGetLastError();
}

hipError_t launch_coef_stats(const SysDesc *dsys, int d, int M, double *part, int nblk,
                             double *out, hipStream_t s) {
  if (d == 3)
    hipLaunchKernelGGL(coef_stats_kernel<3>, dim3(nblk), dim3(NT), 0, s, dsys, part);
  else
    hipLaunchKernelGGL(coef_stats_kernel<2>, dim3(nblk), dim3(NT), 0, s, dsys, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(coef_stats_final_kernel, dim3(1), dim3(NT), 0, s, part, nblk, out);
  return hipGetLastError();
}

}  // namespace csl
