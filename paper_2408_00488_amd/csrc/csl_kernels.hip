// gfx950 kernels of the absolute-value preconditioned MINRES solver
// (arXiv:2408.00488): the persistent multi-system scheduler, the phase tiles
// of one MINRES iteration, stand-alone A and P^{-1} applications, the
// adjoint reduction and the coefficient set-up reductions.
//
// This file is the 256-thread instance (namespace csl::wg256).  It is also
// compiled as two 512-thread instances of the persistent solver alone
// (CSL_SOLVE_ONLY) for systems whose transforms all run on the LDS FFT:
// csl_kernels_wg512.hip for 2-D ones (CSL_2D_FFT_ONLY) and
// csl_kernels_wg512x.hip for either dimension (CSL_FFT_ONLY).  Eight waves
// per workgroup at 128 registers keep twice the waves per CU in flight.
// csl_kernels_wg256h.hip is a 256-thread solver with the FP16 split-product
// sine-matrix engine (CSL_GEMM16) for the systems that use it.
#include <math.h>

#include "csl_device.hpp"
#include "csl_kernels.hpp"

#ifndef CSL_SOLVE_ONLY
#define CSL_SOLVE_ONLY 0
#endif
#ifndef CSL_2D_FFT_ONLY
#define CSL_2D_FFT_ONLY 0
#endif
#ifndef CSL_FFT_ONLY
#define CSL_FFT_ONLY 0
#endif
#ifndef CSL_GEMM16
#define CSL_GEMM16 0
#endif
#ifndef CSL_PLANE
#define CSL_PLANE 0
#endif
#ifndef CSL_PLANE_F64
#define CSL_PLANE_F64 0
#endif
#ifndef CSL_WAVES_PER_EU
#define CSL_WAVES_PER_EU (CSL_NT / 128)
#endif

namespace csl {
namespace CSL_KNS {

template <typename R>
__device__ __forceinline__ Cx<R> to_cx(double2 v) {
  return Cx<R>{(R)v.x, (R)v.y};
}

#if CSL_PLANE
// ---------------------------------------------------------------------------
// Staged stencil rows of phase X (plane instance, 3-D).  The plane phase
// leaves the LDS beyond the row phases' line buffer and twiddles free, so
// phase X copies the rows of zhat_j that a chunk's stencil reads along axes
// 1 and 2 (its rows and the one on either side) into it with the LDS DMA,
// the next chunk's while the current one is transformed and stored; the
// fill loads only zhat's neighbours along axis 0 and the coefficient from
// memory.  The values are the same, so the result is too.
// ---------------------------------------------------------------------------
#define CSL_LDS __attribute__((address_space(3)))

struct XStage {
  int s0, s1;   // staged rows [s0, s1)
};

template <int LDSB>
__device__ __forceinline__ int x_stage_offset() {
  return LDSB + tw_lds_bytes(LDSB);
}

// zhat entries of the staging area: a chunk's rows and one on either side
__device__ __forceinline__ int x_stage_cap(const SysDesc &S) { return (S.lpt_x + 2) * S.n[2]; }

template <int LDSB>
__device__ __forceinline__ bool x_stage_fits(const SysDesc &S) {
  return x_stage_offset<LDSB>() + (long long)x_stage_cap(S) * 16 <= kPlaneLdsBytes;
}

__device__ __forceinline__ XStage x_stage_rows(const SysDesc &S, const LineTile &t) {
  XStage g;
  g.s0 = max(0, t.row0 - 1);
  g.s1 = min(S.rows, t.row0 + t.nl + 1);
  return g;
}

// Start the copy of rows [g.s0, g.s1) of zhat: instruction i of a wave
// moves 16-byte entries 64 i .. 64 i + 63, one per lane, to consecutive LDS
// slots.  Completion is awaited with the vector-memory counter.
__device__ __forceinline__ void x_stage_issue(const SysDesc &S, const CSL_G double2 *zj, char *stage,
                                              XStage g) {
  const int n2 = S.n[2];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nz = (g.s1 - g.s0) * n2;
  double2 *lz = reinterpret_cast<double2 *>(stage);
  const CSL_G double2 *gz = zj + (size_t)g.s0 * n2;
  for (int i = w; i * 64 < nz; i += NT / 64) {
    const int u = i * 64 + lane;
    if (u < nz)
      __builtin_amdgcn_global_load_lds((CSL_G void *)(gz + u), (CSL_LDS void *)(lz + i * 64), 16, 0, 0);
  }
}

// stencil_load<3> with zhat at the point and along axes 1 and 2 read from
// the staged rows; q is the point's entry in them
__device__ __forceinline__ StencilIn<3> stencil_load_staged(const SysDesc &S,
                                                           const CSL_G double2 *__restrict__ u,
                                                           int p, const int (&idx)[3],
                                                           const double2 *lz, int q) {
  StencilIn<3> in;
  const CSL_G double *__restrict__ A = gbl(S.a);
  const int n2 = S.n[2];
  in.c = lz[q];
  in.ap = A[p];
  in.inb = 0u;
  in.ina = 0u;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const bool lo = idx[ax] > 0, hi = idx[ax] < S.n[ax] - 1;
    in.inb |= (lo ? 1u : 0u) << ax;
    in.ina |= (hi ? 1u : 0u) << ax;
    if (ax == 0) {
      const int st = S.st[0];
      in.b[0] = lo ? ldg(u + (p - st)) : make_double2(0.0, 0.0);
      in.a[0] = hi ? ldg(u + (p + st)) : make_double2(0.0, 0.0);
      in.ab[0] = lo ? A[p - st] : 0.0;
      in.aa[0] = hi ? A[p + st] : 0.0;
    } else {
      const int sq = (ax == 1) ? n2 : 1;
      in.b[ax] = lo ? lz[q - sq] : make_double2(0.0, 0.0);
      in.a[ax] = hi ? lz[q + sq] : make_double2(0.0, 0.0);
      in.ab[ax] = lo ? A[p - sq] : 0.0;
      in.aa[ax] = hi ? A[p + sq] : 0.0;
    }
  }
  return in;
}
#endif  // CSL_PLANE

// ---------------------------------------------------------------------------
// K_X, rows of the contiguous axis, always FP64 (it transforms Lanczos
// vectors, not preconditioner data).
//   iter 0: Tv_1 = W_c f; partial ||f||^2; zero the output x.
//   iter j: q = A zhat_j = conj(K zhat_j + conj(lambda) zhat_j) (complex
//           storage of the block product), partial delta_j = <zhat_j, q>,
//           Tq = W_c q.
// ---------------------------------------------------------------------------
template <int D, int LDSB, class E>
__device__ __forceinline__ void tile_X(const SysDesc &S, const IOPtr &io, int iter, int tile, char *smem,
                       double *red) {
  const double *Wm = E::matrix(S, D - 1);
  Cx<double> *buf = reinterpret_cast<Cx<double> *>(smem);
  Cx<double> *twl = reinterpret_cast<Cx<double> *>(smem + LDSB);
  load_twiddles_cached<double>(twl, S.lg[D - 1]);
  double acc = 0.0;
  const int c1 = min(S.nchunk[K_X], (tile + 1) * S.cpt[K_X]);
#if CSL_PLANE
  // staged rows (plane instance): the first chunk's copy starts here
  const bool stg = (D == 3) && S.plane && iter > 0 && x_stage_fits<LDSB>(S);
  char *stage = smem + x_stage_offset<LDSB>();
  if (stg) {
    x_stage_issue(S, gbl(S.Z[iter & 1]), stage,
                  x_stage_rows(S, line_tile(S, D - 1, S.lpt_x, tile * S.cpt[K_X])));
  }
#endif
  for (int chunk = tile * S.cpt[K_X]; chunk < c1; ++chunk) {
    const LineTile t = line_tile(S, D - 1, S.lpt_x, chunk);
    CSL_G Cx<double> *out;
#if CSL_PLANE
    if (stg) {
      const CSL_G double2 *__restrict__ zj = gbl(S.Z[iter & 1]);
      const double al = S.alpha, be = S.beta;
      const XStage g = x_stage_rows(S, t);
      const double2 *lz = reinterpret_cast<const double2 *>(stage);
      const int n2 = S.n[2];
      // this wave's copies (and stores) done, then every wave's
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      E::template fill2<1>(
          buf, t,
          [&](int l, int r, int p) {
            int idx[3];
            row_index<3>(S, t.row0 + l, r, idx);
            return stencil_load_staged(S, zj, p, idx, lz, (t.row0 + l - g.s0) * n2 + r);
          },
          [&](int, int, int, const StencilIn<3> &in) {
            const double2 kz = stencil_apply<3>(S, in);
            const double2 zz = in.c;
            const double qx = kz.x + al * zz.x + be * zz.y;
            const double qy = -(kz.y + al * zz.y - be * zz.x);
            acc += zz.x * qx + zz.y * qy;
            return Cx<double>{qx, qy};
          });
      // the fill ended with a barrier: the staging area is free for the
      // next chunk's rows, which arrive while this chunk is transformed
      if (chunk + 1 < c1)
        x_stage_issue(S, zj, stage, x_stage_rows(S, line_tile(S, D - 1, S.lpt_x, chunk + 1)));
      out = gbl(reinterpret_cast<Cx<double> *>(S.Tq));
    } else
#endif
    if (iter == 0) {
      const CSL_G double2 *__restrict__ f = gbl(io.f);
      CSL_G double2 *__restrict__ X = gbl(io.x);
      E::template fill<4>(buf, t, [&](int, int, int p) {
        const double2 v = ldg(f + p);
        acc += v.x * v.x + v.y * v.y;
        st_nt(X + p, 0.0, 0.0);
        return Cx<double>{v.x, v.y};
      });
      out = gbl(reinterpret_cast<Cx<double> *>(S.Tv[1]));
    } else {
      const CSL_G double2 *__restrict__ zj = gbl(S.Z[iter & 1]);
      const double al = S.alpha, be = S.beta;
      E::template fill2<1>(
          buf, t,
          [&](int l, int r, int p) {
            int idx[3];
            row_index<D>(S, t.row0 + l, r, idx);
            return stencil_load<D>(S, zj, p, idx);
          },
          [&](int, int, int, const StencilIn<D> &in) {
            const double2 kz = stencil_apply<D>(S, in);
            const double2 zz = in.c;
            const double qx = kz.x + al * zz.x + be * zz.y;
            const double qy = -(kz.y + al * zz.y - be * zz.x);
            acc += zz.x * qx + zz.y * qy;
            return Cx<double>{qx, qy};
          });
      out = gbl(reinterpret_cast<Cx<double> *>(S.Tq));
    }
    const Cx<double> *o = E::transform(buf, t, twl, Wm);
#if CSL_PLANE
    if (S.plane) {
      // plane layout: all real parts, then all imaginary parts
      CSL_G double *od = reinterpret_cast<CSL_G double *>(out);
      const int M = S.M;
      E::store_blk(o, t, [&](int, int, int q, Cx<double> v) {
        st_nt(od + q, v.x);
        st_nt(od + M + q, v.y);
      });
      continue;
    }
#endif
    E::store_blk(o, t, [&](int, int, int q, Cx<double> v) { st_nt(out + q, v); });
  }
  const double s = wg_sum(acc, red);
  if (threadIdx.x == 0) S.part[tile] = s;
}

// ---------------------------------------------------------------------------
// Strided passes (columns), preconditioner precision R.
//   First strided pass (2-D K_Y, 3-D K_Y1): input is the new Lanczos vector
//     Tv_{j+1} = Tq - (delta_j/gamma_j) Tv_j - (gamma_j/gamma_{j-1}) Tv_{j-1}
//     (FP64, stored), or Tv_1 at iteration 0.
//   K_Y: forward transform along axis 0, per-mode factor, inverse transform.
//   Last strided pass (2-D K_Y, 3-D K_Y1I): output T' and the partial of
//     gamma_{j+1}^2 = <z_{j+1}, v_{j+1}> = <T', Tv_{j+1}> (W_c orthogonal).
// ---------------------------------------------------------------------------
template <typename R, int D, int LDSB, class E>
__device__ __forceinline__ void tile_Y(const SysDesc &S, int kind, int iter, int tile, char *smem, double *red) {
  Cx<R> *buf = reinterpret_cast<Cx<R> *>(smem);
  const int ax = (kind == K_Y) ? 0 : 1;
  const R *Wm = E::matrix(S, ax);
  Cx<R> *twl = reinterpret_cast<Cx<R> *>(smem + LDSB);
  load_twiddles_cached<R>(twl, S.lg[ax]);
  CSL_G Cx<R> *T = gbl(reinterpret_cast<Cx<R> *>(S.T));
  const bool first = (kind == K_Y1) || (D == 2);
  const int j = iter;
  double gacc = 0.0;
  const int c1 = min(S.nchunk[kind], (tile + 1) * S.cpt[kind]);
  for (int chunk = tile * S.cpt[kind]; chunk < c1; ++chunk) {
  const LineTile t = line_tile(S, ax, S.lpt_s[ax], chunk);
  if (first) {
    if (j == 0) {
      const CSL_G double2 *__restrict__ v1 = gbl(S.Tv[1]);
      E::template fill<4>(buf, t, [&](int, int, int p) { return to_cx<R>(ldg(v1 + p)); });
    } else {
      const Ctl *C = S.ctl;
      const double g = ld_ctl(&C->gamma), go = ld_ctl(&C->gamma_old);
      const double dl = ld_ctl(&C->delta);
      const double cd = dl / g, cg = g / go;
      const CSL_G double2 *__restrict__ tq = gbl(S.Tq);
      const CSL_G double2 *__restrict__ vj = gbl(S.Tv[j & 1]);
      CSL_G double2 *__restrict__ vout = gbl(S.Tv[(j + 1) & 1]);   // holds Tv_{j-1}
      const bool has_vm1 = j >= 2;
      struct In3 {
        double2 q, v1, v0;
      };
      E::template fill2<CSL_U(2)>(
          buf, t,
          [&](int, int, int p) {
            In3 in;
            in.q = ldg(tq + p);
            in.v1 = ldg(vj + p);
            in.v0 = has_vm1 ? ldg(vout + p) : make_double2(0.0, 0.0);
            return in;
          },
          [&](int, int, int p, const In3 &in) {
            const double vx = in.q.x - cd * in.v1.x - cg * in.v0.x;
            const double vy = in.q.y - cd * in.v1.y - cg * in.v0.y;
            st_nt(vout + p, vx, vy);
            return Cx<R>{(R)vx, (R)vy};
          });
    }
  } else {
    E::template fill<4>(buf, t, [&](int, int, int p) { return ldg(T + p); });
  }
  Cx<R> *o = E::transform(buf, t, twl, Wm);
  if (kind == K_Y) {
    const R ab = (sizeof(R) == 8) ? (R)S.abar : (R)S.abar_f;
    const R al = (sizeof(R) == 8) ? (R)S.alpha : (R)S.alpha_f;
    const R be = (sizeof(R) == 8) ? (R)S.beta : (R)S.beta_f;
    const CSL_G R *mu0;
    const CSL_G R *mu1;
    const CSL_G R *mu2;
    if constexpr (sizeof(R) == 8) {
      mu0 = gbl(reinterpret_cast<const R *>(S.mu[0]));
      mu1 = gbl(reinterpret_cast<const R *>(S.mu[1]));
      mu2 = gbl(reinterpret_cast<const R *>(S.mu[2]));
    } else {
      mu0 = gbl(reinterpret_cast<const R *>(S.mu_f[0]));
      mu1 = gbl(reinterpret_cast<const R *>(S.mu_f[1]));
      mu2 = gbl(reinterpret_cast<const R *>(S.mu_f[2]));
    }
    // gamma_{j+1}^2 = <P^{-1} v, v> = sum_k s_k |(W v)_k|^2: here W v is the
    // fully transformed Lanczos vector, so its partial comes from this pass.
    gacc += E::scale_transform(buf, t, twl, Wm, [&](int l, int r) -> R {
      R lam;
      if (D == 2) {
        lam = mu0[r] + mu1[t.c0 + l];
      } else {
        lam = (mu0[r] + mu1[t.outer]) + mu2[t.c0 + l];
      }
      const R sh = ab * lam + al;
      return (R)1 / sqrt(sh * sh + be * be);
    }, &o);
  }
  E::store(o, t, [&](int, int, int p, Cx<R> v) { st_nt(T + p, v); });
  }
  if (kind == K_Y) {
    const double sg = wg_sum(gacc, red);
    if (threadIdx.x == 0) S.part[tile] = sg;
  }
}

// ---------------------------------------------------------------------------
// K_Z, rows of the contiguous axis, precision R: z_{j+1} = W_c T',
// zhat_{j+1} = z_{j+1} / gamma_{j+1}; then the update of step j (j >= 1):
//   w_{j+1} = (zhat_j - e3 w_{j-1} - e2 w_j) / e1,  x_j = x_{j-1} + ceta w_{j+1}
// with x held as its conjugate (the user's z).
// ---------------------------------------------------------------------------
template <typename R, int D, int LDSB, class E>
__device__ __forceinline__ void tile_Z(const SysDesc &S, const IOPtr &io, int iter, int tile, char *smem) {
  const R *Wm = E::matrix(S, D - 1);
  Cx<R> *buf = reinterpret_cast<Cx<R> *>(smem);
  Cx<R> *twl = reinterpret_cast<Cx<R> *>(smem + LDSB);
  const Ctl *C = S.ctl;
  const int j = iter;
  const int mode = j == 0 ? ZM_DEFER : ld_ctl(&C->zmode);
  CSL_G double2 *__restrict__ X = gbl(io.x);
  const int c1 = min(S.nchunk[K_Z], (tile + 1) * S.cpt[K_Z]);
  if (mode == ZM_FLUSH) {
    // the deferred step m = j - 1 alone: w_j = (zhat_{j-1} - e3 w_{j-2} -
    // e2 w_{j-1}) / e1 with step m's coefficients, x += ceta w_j
    const double e1 = ld_ctl(&C->e1), e2 = ld_ctl(&C->e2), e3 = ld_ctl(&C->e3);
    const double ceta = ld_ctl(&C->ceta);
    const double ie1 = 1.0 / e1;
    const CSL_G double2 *__restrict__ zm = gbl(S.Z[(j + 1) & 1]);
    CSL_G double2 *__restrict__ wa = gbl(S.W[j & 1]);          // w_{j-2} -> w_j
    const CSL_G double2 *__restrict__ wb = gbl(S.W[(j + 1) & 1]);   // w_{j-1}
    const bool use_a = j > 3, use_b = j > 2, use_x = j > 2;
    for (int chunk = tile * S.cpt[K_Z]; chunk < c1; ++chunk) {
      const LineTile t = line_tile(S, D - 1, S.lpt_z, chunk);
      const int total = tile_elems(t);
      for (int e = threadIdx.x; e < total; e += NT) {
        int l, r;
        if (!split_elem(t, e, l, r)) continue;
        const int p = t.base + l * t.lstride + r * t.stride;
        const double2 z = ldg(zm + p);
        const double2 w0 = use_a ? ldg(wa + p) : make_double2(0.0, 0.0);
        const double2 w1 = use_b ? ldg(wb + p) : make_double2(0.0, 0.0);
        const double2 x = use_x ? ldg(X + p) : make_double2(0.0, 0.0);
        const double wx = (z.x - e3 * w0.x - e2 * w1.x) * ie1;
        const double wy = (z.y - e3 * w0.y - e2 * w1.y) * ie1;
        st_nt(wa + p, wx, wy);
        st_nt(X + p, x.x + ceta * wx, x.y - ceta * wy);
      }
    }
    return;
  }
  load_twiddles_cached<R>(twl, S.lg[D - 1]);
  const CSL_G Cx<R> *T = gbl(reinterpret_cast<const Cx<R> *>(S.T));
  const double g = ld_ctl(&C->gamma);
  const bool store_z = (g != 0.0);
  const double ig = store_z ? 1.0 / g : 0.0;
  CSL_G double2 *__restrict__ znew = gbl(S.Z[(j + 1) & 1]);
  for (int chunk = tile * S.cpt[K_Z]; chunk < c1; ++chunk) {
  const LineTile t = line_tile(S, D - 1, S.lpt_z, chunk);
#if CSL_PLANE
  if (S.plane) {
    // plane layout: all real parts, then all imaginary parts
    const CSL_G R *Tr = reinterpret_cast<const CSL_G R *>(T);
    const int M = S.M;
    E::template fill_blk<CSL_U(8)>(buf, t, [&](int, int, int q) { return Cx<R>{Tr[q], Tr[M + q]}; });
  } else
#endif
  E::template fill_blk<CSL_U(8)>(buf, t, [&](int, int, int q) { return ldg(T + q); });
  const Cx<R> *o = E::transform(buf, t, twl, Wm);
  if (mode == ZM_DEFER) {
    E::store(o, t, [&](int, int, int p, Cx<R> v) {
      st_nt(znew + p, (double)v.x * ig, (double)v.y * ig);
    });
    continue;
  }
  const double e1 = ld_ctl(&C->e1), e2 = ld_ctl(&C->e2), e3 = ld_ctl(&C->e3);
  const double ceta = ld_ctl(&C->ceta);
  const double ie1 = 1.0 / e1;
  const CSL_G double2 *__restrict__ zj = gbl(S.Z[j & 1]);
  if (mode == ZM_SINGLE) {
    CSL_G double2 *__restrict__ wnew = gbl(S.W[(j + 1) & 1]);   // holds w_{j-1} before the update
    const CSL_G double2 *__restrict__ wj = gbl(S.W[j & 1]);
    const bool use_wm1 = j > 2, use_wj = j > 1, use_x = j > 1;
    struct In4 {
      double2 z, w0, w1, x;
    };
    E::template store2<CSL_U(2)>(
        o, t,
        [&](int p) {
          In4 in;
          in.z = ldg(zj + p);
          in.w0 = use_wm1 ? ldg(wnew + p) : make_double2(0.0, 0.0);
          in.w1 = use_wj ? ldg(wj + p) : make_double2(0.0, 0.0);
          in.x = use_x ? ldg(X + p) : make_double2(0.0, 0.0);
          return in;
        },
        [&](int p, Cx<R> v, const In4 &in) {
          if (store_z) st_nt(znew + p, (double)v.x * ig, (double)v.y * ig);
          const double wx = (in.z.x - e3 * in.w0.x - e2 * in.w1.x) * ie1;
          const double wy = (in.z.y - e3 * in.w0.y - e2 * in.w1.y) * ie1;
          st_nt(wnew + p, wx, wy);
          st_nt(X + p, in.x.x + ceta * wx, in.x.y - ceta * wy);
        });
    continue;
  }
  // ZM_PAIR: steps j-1 (deferred, coefficients e*p) and j:
  //   w_j     = (zhat_{j-1} - e3p w_{j-2} - e2p w_{j-1}) / e1p
  //   w_{j+1} = (zhat_j     - e3  w_{j-1} - e2  w_j    ) / e1
  //   x += cetap w_j, then x += ceta w_{j+1}
  // zhat_{j-1} sits in the buffer that receives zhat_{j+1}, w_{j-2} in the
  // one that receives w_j: each entry is read before it is overwritten by
  // the same thread.
  const double e1p = ld_ctl(&C->e1p), e2p = ld_ctl(&C->e2p), e3p = ld_ctl(&C->e3p);
  const double cetap = ld_ctl(&C->cetap);
  const double ie1p = 1.0 / e1p;
  CSL_G double2 *__restrict__ wa = gbl(S.W[j & 1]);           // w_{j-2} -> w_j
  CSL_G double2 *__restrict__ wb = gbl(S.W[(j + 1) & 1]);     // w_{j-1} -> w_{j+1}
  const bool use_a = j > 3, use_b = j > 2, use_x = j > 2;
  struct In5 {
    double2 zm, z, wa, wb, x;
  };
  E::template store2<1>(
      o, t,
      [&](int p) {
        In5 in;
        in.zm = ldg(znew + p);   // zhat_{j-1}
        in.z = ldg(zj + p);
        in.wa = use_a ? ldg(wa + p) : make_double2(0.0, 0.0);
        in.wb = use_b ? ldg(wb + p) : make_double2(0.0, 0.0);
        in.x = use_x ? ldg(X + p) : make_double2(0.0, 0.0);
        return in;
      },
      [&](int p, Cx<R> v, const In5 &in) {
        if (store_z) st_nt(znew + p, (double)v.x * ig, (double)v.y * ig);
        const double ax = (in.zm.x - e3p * in.wa.x - e2p * in.wb.x) * ie1p;
        const double ay = (in.zm.y - e3p * in.wa.y - e2p * in.wb.y) * ie1p;
        const double bx = (in.z.x - e3 * in.wb.x - e2 * ax) * ie1;
        const double by = (in.z.y - e3 * in.wb.y - e2 * ay) * ie1;
        st_nt(wa + p, ax, ay);
        st_nt(wb + p, bx, by);
        const double xx = in.x.x + cetap * ax, xy = in.x.y - cetap * ay;
        st_nt(X + p, xx + ceta * bx, xy - ceta * by);
      });
  }
}

// True residual partial ||f - (K + lambda I) z||^2 with z the user output.
template <int D>
__device__ __forceinline__ void tile_PR(const SysDesc &S, const IOPtr &io, int tile, double *red) {
  const int nlast = S.n[D - 1];
  const int r0 = tile * S.cpt[K_PR] * S.rpt;
  const int r1 = min(S.rows, r0 + S.cpt[K_PR] * S.rpt);
  const int p0 = r0 * nlast, p1 = r1 * nlast;
  const CSL_G double2 *__restrict__ X = gbl(io.x);
  const CSL_G double2 *__restrict__ f = gbl(io.f);
  const double al = S.alpha, be = S.beta;
  double acc = 0.0;
  for (int p = p0 + (int)threadIdx.x; p < p1; p += NT) {
    const int row = p / nlast;
    int idx[3];
    row_index<D>(S, row, p - row * nlast, idx);
    const double2 kx = stencil_K<D>(S, X, p, idx);
    const double2 xv = ldg(X + p);
    const double ux = kx.x + al * xv.x - be * xv.y;
    const double uy = kx.y + al * xv.y + be * xv.x;
    const double2 fv = ldg(f + p);
    const double rx = fv.x - ux, ry = fv.y - uy;
    acc += rx * rx + ry * ry;
  }
  const double s = wg_sum(acc, red);
  if (threadIdx.x == 0) S.part[tile] = s;
}

#if CSL_PLANE
// ---------------------------------------------------------------------------
// Plane phase (3-D, FFT on axes 0 and 1): tile 2c + comp is the real (comp
// 0) or the imaginary (comp 1) part of the plane of contiguous-axis index c,
// a real plane held in LDS in the preconditioner precision (FP32 here on
// 1024 threads, FP64 on 512: an FP64 plane of 127 x 127 leaves LDS for the
// line buffers of eight waves only).  Tq, Tv and T hold
// all real parts, then all imaginary parts, each with plane c contiguous
// (block width one).  In one pass over it:
//   Tv_{j+1} = Tq - (delta_j/gamma_j) Tv_j - (gamma_j/gamma_{j-1}) Tv_{j-1}
//     (FP64, stored; Tv_1 at iteration 0), rounded into the plane;
//   the forward transforms of the axis-1 lines, then of the axis-0 lines
//     with the per-mode factor and the partial of gamma_{j+1}^2, their
//     inverses, then the inverses of the axis-1 lines;
//   T' written once.
// The sine transforms and the per-mode factors are real, so the two parts
// of a plane are transformed independently, and every CU has a plane tile
// (2 n2 of them).  Inside a tile two real lines make one complex line (the
// first its real part, the second its imaginary part); the transformed
// complex line holds their two results the same way.  The values are those
// of the three strided phases (K_Y1, K_Y, K_Y1I) with their intermediate
// kept in LDS instead of T.
//
// Each wave transforms whole lines on its own (wave_fft_line): a wave holds
// 256/L complex lines of the odd extension and exchanges values between
// stages through its own 2 KiB (FP64: 4 KiB) of LDS with no workgroup
// barrier.
// ---------------------------------------------------------------------------
constexpr int kPlaneWaveElts = 256;   // complex values per wave buffer

// Odd extension of the complex line made of real lines la and lb (lb absent:
// zero imaginary part), n = L/2 - 1 points at stride ldp.
template <typename R>
__device__ __forceinline__ Cx<R> pair_ext(const R *la, const R *lb, bool hasb, int ldp, int m, int L,
                                          bool act) {
  const int N = L >> 1;
  if (!act || m == 0 || m == N) return Cx<R>{(R)0, (R)0};
  const int r = m < N ? m - 1 : L - 1 - m;
  const R re = la[r * ldp];
  const R im = hasb ? lb[r * ldp] : (R)0;
  return m < N ? Cx<R>{re, im} : Cx<R>{-re, -im};
}

// Sine transform, in place, of the nlines real lines of a real plane (line l
// at pl[l ldl + r ldp]), lines 2p and 2p + 1 as one complex line.  With
// contiguous lines (ldp = 1) a wave's lines of one round are the plane
// elements [e0, e1): pre(e0, e1) runs before the wave reads them (it may
// write them) and post(e0, e1) after it has written their transforms, each
// on the wave's own lanes.
struct PlaneNoHook {
  __device__ __forceinline__ void operator()(int, int) const {}
};
template <typename R, class Pre = PlaneNoHook, class Post = PlaneNoHook>
__device__ __forceinline__ void plane_dst_pairs(R *pl, Cx<R> *wbuf, const Cx<R> *twl, int nlines, int lg,
                                                int ldl, int ldp, Pre &&pre = Pre(),
                                                Post &&post = Post()) {
  const int L = 1 << lg, Q = L >> 2, N = L >> 1;
  const int G = 64 >> (lg - 2);   // complex lines per wave
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int g = t >> (lg - 2), j = t & (Q - 1);
  Cx<R> *wb = wbuf + w * kPlaneWaveElts;
  const int lo = g * L;
  const R cf = (R)1 / sqrt((R)L);
  const int npairs = (nlines + 1) >> 1;
  for (int p0 = w * G; p0 < npairs; p0 += (NT / 64) * G) {
    const int p = p0 + g;
    const bool act = p < npairs;
    const bool hasb = act && 2 * p + 1 < nlines;
    const int e0 = 2 * p0 * ldl, e1 = min(2 * (p0 + G), nlines) * ldl;
    pre(e0, e1);
    wave_lds_sync();
    R *la = pl + (size_t)(act ? 2 * p : 0) * ldl;
    R *lb = la + ldl;
    Cx<R> a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = pair_ext<R>(la, lb, hasb, ldp, j + q * Q, L, act);
    wave_fft_line<R>(a, wb, lo, j, lg, twl, true);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = j + q * Q;
      if (act && k >= 1 && k < N) {
        const Cx<R> v = dst_out(a[q], cf);
        la[(k - 1) * ldp] = v.x;
        if (hasb) lb[(k - 1) * ldp] = v.y;
      }
    }
    wave_lds_sync();
    post(e0, e1);
  }
}

// FP64 plane: each sine transform of n = N - 1 points runs as a complex FFT
// of N points instead of the 2N points of the odd extension.  With
// S_k = sum_j x_j sin(pi j k / N) and the FFT Y of
//   y_j = sin(pi j / N) (x_j + x_{N-j}) + (x_j - x_{N-j}) / 2   (y_0 = 0),
// Y_m = (S_{2m+1} - S_{2m-1}) - i S_{2m}, and Y_{N-m} the same with +i; so
//   S_{2m}   = i (Y_m - Y_{N-m}) / 2,
//   S_{2m+1} = S_{2m-1} + (Y_m + Y_{N-m}) / 2,   S_1 = Y_0 / 2,
// which holds for complex x as well (every step is linear with real
// coefficients apart from the factor i).  The odd outputs are a running sum
// over m; in FP64 its rounding stays at the level of the FFT's (a few units
// in the last place over 64 terms), while in FP32 it would not, so the FP32
// plane keeps the odd extension.  A line takes Q = N/4 lanes of the wave,
// lane j holding inputs and FFT outputs j + q Q, and after the combination
// the four orthonormal outputs X_{4j} .. X_{4j+3} (X_k = sqrt(2/N) S_k).

// sin(pi i / N) for the lane's inputs i = j + q Q, from the FP64 twiddle
// table (-Im exp(-2 pi i m / TWN) at m = i TWN / (2N))
__device__ __forceinline__ void half_sines(double (&sn)[4], int j, int lgN) {
  const CSL_G Cx<double> *tw = gbl(twiddles<double>());
  const int Q = (1 << lgN) >> 2, step = TWN >> (lgN + 1);
#pragma unroll
  for (int q = 0; q < 4; ++q) sn[q] = -tw[(j + q * Q) * step].y;
}

// y_i of the complex line made of real lines la and lb (lb absent: zero
// imaginary part), x_i at row i - 1 with stride ldp
__device__ __forceinline__ Cx<double> half_in(const double *la, const double *lb, bool hasb, int ldp,
                                              int i, int N, bool act, double sn) {
  if (!act || i == 0) return Cx<double>{0.0, 0.0};
  const int r = i - 1, rr = N - 1 - i;
  const double pa = la[r * ldp], qa = la[rr * ldp];
  const double pb = hasb ? lb[r * ldp] : 0.0, qb = hasb ? lb[rr * ldp] : 0.0;
  return Cx<double>{sn * (pa + qa) + 0.5 * (pa - qa), sn * (pb + qb) + 0.5 * (pb - qb)};
}

// The same from a line held in natural order in the wave buffer (x_i at
// wb[lo + i], i = 1 .. N - 1)
__device__ __forceinline__ Cx<double> half_in_buf(const Cx<double> *wb, int lo, int i, int N, double sn) {
  if (i == 0) return Cx<double>{0.0, 0.0};
  const Cx<double> p = wb[lo + i], q = wb[lo + N - i];
  return Cx<double>{sn * (p.x + q.x) + 0.5 * (p.x - q.x), sn * (p.y + q.y) + 0.5 * (p.y - q.y)};
}

// From the FFT outputs (a[q] = Y_{j + q Q}) to the orthonormal outputs
// x[u] = X_{4j+u} (x[0] is no output for j = 0): the outputs pass through
// the wave buffer to meet Y_{N-m}, and the running sum of the odd outputs is
// a scan over the Q lanes of the line.
__device__ __forceinline__ void half_out(const Cx<double> (&a)[4], Cx<double> *wb, int lo, int j, int lgN,
                                         double cf, Cx<double> (&x)[4]) {
  const int N = 1 << lgN, Q = N >> 2;
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < 4; ++q) wb[lo + j + q * Q] = a[q];
  wave_lds_sync();
  const Cx<double> ya = wb[lo + 2 * j], yb = wb[lo + 2 * j + 1];
  const Cx<double> za = wb[lo + ((N - 2 * j) & (N - 1))], zb = wb[lo + N - 2 * j - 1];
  // (Y_m + Y_{N-m}) / 2 and i (Y_m - Y_{N-m}) / 2 for m = 2j, 2j + 1, times 2 cf
  const Cx<double> ba = j == 0 ? Cx<double>{cf * ya.x, cf * ya.y}
                               : Cx<double>{cf * (ya.x + za.x), cf * (ya.y + za.y)};
  const Cx<double> bb = {cf * (yb.x + zb.x), cf * (yb.y + zb.y)};
  const Cx<double> ea = {-cf * (ya.y - za.y), cf * (ya.x - za.x)};
  const Cx<double> eb = {-cf * (yb.y - zb.y), cf * (yb.x - zb.x)};
  const Cx<double> c = {ba.x + bb.x, ba.y + bb.y};
  // inclusive scan of c over the line's lanes
  Cx<double> in = c;
  for (int d = 1; d < Q; d <<= 1) {
    const double ux = __shfl_up(in.x, (unsigned)d, Q), uy = __shfl_up(in.y, (unsigned)d, Q);
    if (j >= d) {
      in.x += ux;
      in.y += uy;
    }
  }
  const Cx<double> e = {in.x - c.x, in.y - c.y};   // sum over the lanes before this one
  x[0] = ea;
  x[1] = Cx<double>{e.x + ba.x, e.y + ba.y};
  x[2] = eb;
  x[3] = in;
}

// Sine transform, in place, of the nlines real FP64 lines of a plane (line l
// at pl[l ldl + r ldp]) through FFTs of N = 2^lgN points, lines 2p and 2p + 1
// as one complex line.
template <class Pre = PlaneNoHook, class Post = PlaneNoHook>
__device__ __forceinline__ void plane_dst_pairs_half(double *pl, Cx<double> *wbuf, const Cx<double> *twl,
                                                     int nlines, int lgN, int ldl, int ldp,
                                                     Pre &&pre = Pre(), Post &&post = Post()) {
  const int N = 1 << lgN, Q = N >> 2;
  const int G = 64 >> (lgN - 2);   // complex lines per wave
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int g = t >> (lgN - 2), j = t & (Q - 1);
  Cx<double> *wb = wbuf + w * kPlaneWaveElts;
  const int lo = g * N;
  const double cf = 1.0 / sqrt((double)(2 * N));
  double sn[4];
  half_sines(sn, j, lgN);
  const int npairs = (nlines + 1) >> 1;
  for (int p0 = w * G; p0 < npairs; p0 += (NT / 64) * G) {
    const int p = p0 + g;
    const bool act = p < npairs;
    const bool hasb = act && 2 * p + 1 < nlines;
    const int e0 = 2 * p0 * ldl, e1 = min(2 * (p0 + G), nlines) * ldl;
    pre(e0, e1);
    wave_lds_sync();
    double *la = pl + (size_t)(act ? 2 * p : 0) * ldl;
    double *lb = la + ldl;
    Cx<double> a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = half_in(la, lb, hasb, ldp, j + q * Q, N, act, sn[q]);
    wave_fft_line<double>(a, wb, lo, j, lgN, twl, true);
    Cx<double> x[4];
    half_out(a, wb, lo, j, lgN, cf, x);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 4 * j + u;
      if (act && k >= 1) {
        la[(k - 1) * ldp] = x[u].x;
        if (hasb) lb[(k - 1) * ldp] = x[u].y;
      }
    }
    wave_lds_sync();
    post(e0, e1);
  }
}

// Phase X of a plane solve after its first iteration, with rows of n2 = N - 1
// <= 127 points: every row is formed and transformed by one wave on its own
// (G = 256 / N rows a wave, the FP64 transform of N points above), so the
// stencil loads of some waves run under the transforms of others; the
// round's outputs pass through the wave buffers to be stored row-fastest in
// the plane layout.  (Staging a round's rows of zhat by the LDS DMA, as
// tile_X does, changed its time by less than 0.5%.)  Same values as tile_X
// up to the transform's rounding.
template <int LDSB>
__device__ __forceinline__ void tile_XW(const SysDesc &S, int iter, int tile, char *smem, double *red) {
  constexpr int W = NT / 64;
  const int n2 = S.n[2], N = n2 + 1, lgN = S.lg[2] - 1, Q = N >> 2;
  const int G = 64 >> (lgN - 2);
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int g = t >> (lgN - 2), j = t & (Q - 1);
  Cx<double> *wbase = reinterpret_cast<Cx<double> *>(smem);
  Cx<double> *wb = wbase + w * kPlaneWaveElts;
  Cx<double> *twl = reinterpret_cast<Cx<double> *>(smem + LDSB);
  load_twiddles_cached<double>(twl, lgN);
  const int lo = g * N;
  const double cf = 1.0 / sqrt((double)(2 * N));
  double sn[4];
  half_sines(sn, j, lgN);
  const CSL_G double2 *__restrict__ zj = gbl(S.Z[iter & 1]);
  const double al = S.alpha, be = S.beta;
  CSL_G double *__restrict__ od = reinterpret_cast<CSL_G double *>(gbl(S.Tq));
  const int M = S.M, rows = S.rows;
  const int r_begin = tile * S.cpt[K_X] * S.lpt_x;
  const int r_end = min(rows, (tile + 1) * S.cpt[K_X] * S.lpt_x);
  double acc = 0.0;
  for (int rb = r_begin; rb < r_end; rb += G * W) {
    const int row = rb + w * G + g;
    const bool act = row < r_end;
    Cx<double> x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = j + q * Q;
      x[q] = Cx<double>{0.0, 0.0};
      if (act && i >= 1) {
        int idx[3];
        row_index<3>(S, row, i - 1, idx);
        const int p = row * n2 + i - 1;
        const StencilIn<3> in = stencil_load<3>(S, zj, p, idx);
        const double2 kz = stencil_apply<3>(S, in);
        const double2 zz = in.c;
        const double qx = kz.x + al * zz.x + be * zz.y;
        const double qy = -(kz.y + al * zz.y - be * zz.x);
        acc += zz.x * qx + zz.y * qy;
        x[q] = Cx<double>{qx, qy};
      }
    }
    // the line in natural order, then its combined input
#pragma unroll
    for (int q = 0; q < 4; ++q) wb[lo + j + q * Q] = x[q];
    wave_lds_sync();
    Cx<double> a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = half_in_buf(wb, lo, j + q * Q, N, sn[q]);
    wave_fft_line<double>(a, wb, lo, j, lgN, twl, true);
    half_out(a, wb, lo, j, lgN, cf, x);
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 4 * j + u;
      if (k >= 1) wb[g * n2 + k - 1] = x[u];
    }
    __syncthreads();
    // rows fastest: for each output k the round's rows are consecutive
    const int R = min(G * W, r_end - rb);
    for (int e = threadIdx.x; e < R * n2; e += NT) {
      const int k = e / R, rr = e - k * R;
      const Cx<double> v = wbase[(rr / G) * kPlaneWaveElts + (rr % G) * n2 + k];
      const int q = k * rows + rb + rr;
      st_nt(od + q, v.x);
      st_nt(od + M + q, v.y);
    }
    __syncthreads();
  }
  const double s = wg_sum(acc, red);
  if (threadIdx.x == 0) S.part[tile] = s;
}

// Phase Z of a plane solve with rows of n2 = N - 1 <= 127 points, per wave as
// tile_XW: a round's rows of T' (plane layout) are read rows-fastest into LDS,
// then every wave transforms its rows (FP32: the odd extension, 128 / N rows
// a wave; FP64: FFTs of N points, 256 / N rows a wave) and applies the step's
// update to its outputs itself, so the update's loads and stores of some
// waves run under the transforms of others.  Same values as tile_Z up to the
// transform's rounding; the flush of a deferred step (no transform) is
// tile_Z's.
template <typename R, int LDSB>
__device__ __forceinline__ void tile_ZW(const SysDesc &S, const IOPtr &io, int iter, int tile, char *smem) {
  constexpr int W = NT / 64;
  constexpr bool kHalf = sizeof(R) == 8;
  const Ctl *C = S.ctl;
  const int j = iter;
  const int mode = j == 0 ? ZM_DEFER : ld_ctl(&C->zmode);
  if (mode == ZM_FLUSH) {
    tile_Z<R, 3, LDSB, FftEng<R, LDSB>>(S, io, iter, tile, smem);
    return;
  }
  const int n2 = S.n[2], N = n2 + 1;
  const int lgF = kHalf ? S.lg[2] - 1 : S.lg[2];   // FFT of N (FP64) or 2N (FP32) points
  const int F = 1 << lgF, Q = F >> 2;
  const int G = 64 >> (lgF - 2);
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int g = t >> (lgF - 2), jl = t & (Q - 1);
  Cx<R> *wb = reinterpret_cast<Cx<R> *>(smem) + w * kPlaneWaveElts;
  // the round's rows of T', row-major, after the wave buffers
  Cx<R> *tin = reinterpret_cast<Cx<R> *>(smem) + W * kPlaneWaveElts;
  Cx<R> *twl = reinterpret_cast<Cx<R> *>(smem + LDSB);
  load_twiddles_cached<R>(twl, lgF);
  const int lo = g * F;
  const R cf = (R)1 / sqrt((R)(kHalf ? 2 * N : F));
  double sn[4];
  if constexpr (kHalf) half_sines(sn, jl, lgF);
  const CSL_G R *__restrict__ Tr = reinterpret_cast<const CSL_G R *>(gbl(S.T));
  const int M = S.M, rows = S.rows;
  const int r_begin = tile * S.cpt[K_Z] * S.lpt_z;
  const int r_end = min(rows, (tile + 1) * S.cpt[K_Z] * S.lpt_z);
  const double g2 = ld_ctl(&C->gamma);
  const bool store_z = (g2 != 0.0);
  const double ig = store_z ? 1.0 / g2 : 0.0;
  CSL_G double2 *__restrict__ X = gbl(io.x);
  CSL_G double2 *__restrict__ znew = gbl(S.Z[(j + 1) & 1]);
  const CSL_G double2 *__restrict__ zj = gbl(S.Z[j & 1]);
  double e1 = 0, e2 = 0, e3 = 0, ceta = 0, ie1 = 0, e2p = 0, e3p = 0, cetap = 0, ie1p = 0;
  if (mode != ZM_DEFER) {
    e1 = ld_ctl(&C->e1);
    e2 = ld_ctl(&C->e2);
    e3 = ld_ctl(&C->e3);
    ceta = ld_ctl(&C->ceta);
    ie1 = 1.0 / e1;
  }
  if (mode == ZM_PAIR) {
    e2p = ld_ctl(&C->e2p);
    e3p = ld_ctl(&C->e3p);
    cetap = ld_ctl(&C->cetap);
    ie1p = 1.0 / ld_ctl(&C->e1p);
  }
  // ZM_SINGLE: wn holds w_{j-1} and receives w_{j+1}, wo holds w_j;
  // ZM_PAIR: wo holds w_{j-2} and receives w_j, wn holds w_{j-1} and
  // receives w_{j+1} (each entry read before the same lane overwrites it)
  CSL_G double2 *__restrict__ wo = gbl(S.W[j & 1]);
  CSL_G double2 *__restrict__ wn = gbl(S.W[(j + 1) & 1]);
  auto update = [&](int p, Cx<R> v) {
    if (mode == ZM_DEFER) {
      st_nt(znew + p, (double)v.x * ig, (double)v.y * ig);
    } else if (mode == ZM_SINGLE) {
      const double2 z = ldg(zj + p);
      const double2 w0 = j > 2 ? ldg(wn + p) : make_double2(0.0, 0.0);
      const double2 w1 = j > 1 ? ldg(wo + p) : make_double2(0.0, 0.0);
      const double2 x = j > 1 ? ldg(X + p) : make_double2(0.0, 0.0);
      if (store_z) st_nt(znew + p, (double)v.x * ig, (double)v.y * ig);
      const double wx = (z.x - e3 * w0.x - e2 * w1.x) * ie1;
      const double wy = (z.y - e3 * w0.y - e2 * w1.y) * ie1;
      st_nt(wn + p, wx, wy);
      st_nt(X + p, x.x + ceta * wx, x.y - ceta * wy);
    } else {
      const double2 zm = ldg(znew + p);   // zhat_{j-1}
      const double2 z = ldg(zj + p);
      const double2 wa = j > 3 ? ldg(wo + p) : make_double2(0.0, 0.0);
      const double2 wbv = j > 2 ? ldg(wn + p) : make_double2(0.0, 0.0);
      const double2 x = j > 2 ? ldg(X + p) : make_double2(0.0, 0.0);
      if (store_z) st_nt(znew + p, (double)v.x * ig, (double)v.y * ig);
      const double ax = (zm.x - e3p * wa.x - e2p * wbv.x) * ie1p;
      const double ay = (zm.y - e3p * wa.y - e2p * wbv.y) * ie1p;
      const double bx = (z.x - e3 * wbv.x - e2 * ax) * ie1;
      const double by = (z.y - e3 * wbv.y - e2 * ay) * ie1;
      st_nt(wo + p, ax, ay);
      st_nt(wn + p, bx, by);
      const double xx = x.x + cetap * ax, xy = x.y - cetap * ay;
      st_nt(X + p, xx + ceta * bx, xy - ceta * by);
    }
  };
  for (int rb = r_begin; rb < r_end; rb += G * W) {
    const int R_ = min(G * W, r_end - rb);
    for (int e = threadIdx.x; e < R_ * n2; e += NT) {
      const int k = e / R_, rr = e - k * R_;
      const int q = k * rows + rb + rr;
      tin[rr * n2 + k] = Cx<R>{Tr[q], Tr[M + q]};
    }
    __syncthreads();
    const int rr = w * G + g;
    const int row = rb + rr;
    const bool act = row < r_end;
    const Cx<R> *xl = tin + (act ? rr : 0) * n2;
    Cx<R> a[4];
    if constexpr (kHalf) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = jl + q * Q;
        a[q] = Cx<R>{0, 0};
        if (act && i >= 1) {
          const Cx<R> u = xl[i - 1], v = xl[N - 1 - i];
          a[q] = Cx<R>{sn[q] * (u.x + v.x) + 0.5 * (u.x - v.x), sn[q] * (u.y + v.y) + 0.5 * (u.y - v.y)};
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = jl + q * Q;
        a[q] = Cx<R>{0, 0};
        if (act && m != 0 && m != N) {
          const Cx<R> u = xl[m < N ? m - 1 : F - 1 - m];
          a[q] = m < N ? u : Cx<R>{-u.x, -u.y};
        }
      }
    }
    __syncthreads();   // every wave has its input: the next round may refill tin
    wave_fft_line<R>(a, wb, lo, jl, lgF, twl, true);
    if constexpr (kHalf) {
      // a lane leaves half_out with four consecutive outputs: back through
      // the wave buffer so that neighbouring lanes update neighbouring points
      Cx<double> x[4];
      half_out(a, wb, lo, jl, lgF, cf, x);
      wave_lds_sync();
#pragma unroll
      for (int u = 0; u < 4; ++u) wb[lo + 4 * jl + u] = x[u];
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = jl + q * Q;
        if (act && k >= 1) update(row * n2 + k - 1, wb[lo + k]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = jl + q * Q;
        if (act && k >= 1 && k < N) update(row * n2 + k - 1, dst_out(a[q], cf));
      }
    }
  }
}

// The plane tile: one part of one plane, in the preconditioner precision R
// (FP32 in the 1024-thread instance, FP64 in the 512-thread one).
template <typename R>
__device__ __forceinline__ void tile_YP(const SysDesc &S, int iter, int tile, char *smem,
                                        double *red) {
  const int n0 = S.n[0], n1 = S.n[1];
  const int rows = S.rows;
  const int c = tile >> 1, comp = tile & 1;
  R *pl = reinterpret_cast<R *>(smem);
  const size_t pb = ((size_t)rows * sizeof(R) + 127) & ~(size_t)127;
  Cx<R> *wbuf = reinterpret_cast<Cx<R> *>(smem + pb);
  // FFT lengths: the odd extension (2 (n + 1)) in FP32, n + 1 in FP64
  constexpr bool kHalf = sizeof(R) == 8;
  const int lg0 = S.lg[0] - (kHalf ? 1 : 0), lg1 = S.lg[1] - (kHalf ? 1 : 0);
  Cx<R> *tw0 = wbuf + (NT / 64) * kPlaneWaveElts;
  // one table when both axes have the same length
  Cx<R> *tw1 = lg1 == lg0 ? tw0 : tw0 + ((1 << lg0) >> 2);
  // the line buffer's twiddle cache lies inside the plane: restage later
  if (threadIdx.x == 0) s_twkey = -1;
  load_twiddles<R>(tw0, lg0);
  if (lg1 != lg0) load_twiddles<R>(tw1, lg1);
  const size_t off = (size_t)comp * S.M + (size_t)c * rows;
  const int j = iter;
  const int lane = threadIdx.x & 63;
  // the plane's rows, each wave its own just before it transforms them:
  // Tv_1 at iteration 0, else the Lanczos update
  const CSL_G double *__restrict__ v1 = reinterpret_cast<const CSL_G double *>(gbl(S.Tv[1])) + off;
  const CSL_G double *__restrict__ tq = reinterpret_cast<const CSL_G double *>(gbl(S.Tq)) + off;
  const CSL_G double *__restrict__ vj = reinterpret_cast<const CSL_G double *>(gbl(S.Tv[j & 1])) + off;
  // holds Tv_{j-1}
  CSL_G double *__restrict__ vout = reinterpret_cast<CSL_G double *>(gbl(S.Tv[(j + 1) & 1])) + off;
  double cd = 0.0, cg = 0.0;
  if (j > 0) {
    const Ctl *C = S.ctl;
    const double g = ld_ctl(&C->gamma), go = ld_ctl(&C->gamma_old);
    const double dl = ld_ctl(&C->delta);
    cd = dl / g;
    cg = g / go;
  }
  const bool has_vm1 = j >= 2;
  auto fill = [&](int e0, int e1) {
    constexpr int U = 4;
    for (int b = e0; b < e1; b += 64 * U) {
      double q[U], a1[U], a0[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = b + u * 64 + lane;
        if (e < e1) {
          if (j == 0) {
            q[u] = v1[e];
          } else {
            q[u] = tq[e];
            a1[u] = vj[e];
            a0[u] = has_vm1 ? vout[e] : 0.0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = b + u * 64 + lane;
        if (e < e1) {
          if (j == 0) {
            pl[e] = (R)q[u];
          } else {
            const double v = q[u] - cd * a1[u] - cg * a0[u];
            st_nt(vout + e, v);
            pl[e] = (R)v;
          }
        }
      }
    }
  };
  // axis 1 forward: n0 lines of n1 points, contiguous in the plane
  if constexpr (kHalf) plane_dst_pairs_half(pl, wbuf, tw1, n0, lg1, n1, 1, fill);
  else plane_dst_pairs<R>(pl, wbuf, tw1, n0, lg1, n1, 1, fill);
  __syncthreads();
  // axis 0: n1 lines of n0 points at stride n1, neighbouring columns in
  // pairs; forward transform, the per-mode factor of each column's own mode
  // with the partial of gamma^2, and the inverse, the scaled modes staying
  // in registers as the inverse's input (the factor of mode k applied to
  // output k and, by the odd symmetry, to output L - k)
  double gacc = 0.0;
  if constexpr (kHalf) {
    // FP64: forward transform of a column pair, the factor of each column's
    // mode with the partial of gamma^2 on the lane's four modes 4 jl .. 4 jl
    // + 3, the scaled modes back through the wave buffer in natural order as
    // the inverse's input, the inverse
    const int N = 1 << lg0, Q = N >> 2;
    const int G = 64 >> (lg0 - 2);
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
    const int g = t >> (lg0 - 2), jl = t & (Q - 1);
    Cx<double> *wb = reinterpret_cast<Cx<double> *>(wbuf) + w * kPlaneWaveElts;
    const int lo = g * N;
    const double ab = S.abar, al = S.alpha, be = S.beta;
    const CSL_G double *mu0 = gbl(S.mu[0]);
    const CSL_G double *mu1 = gbl(S.mu[1]);
    const double m2 = gbl(S.mu[2])[c];
    const double cf = 1.0 / sqrt((double)(2 * N));
    const Cx<double> *twl = reinterpret_cast<const Cx<double> *>(tw0);
    double sn[4], m0[4];
    half_sines(sn, jl, lg0);
#pragma unroll
    for (int u = 0; u < 4; ++u) m0[u] = 4 * jl + u >= 1 ? mu0[4 * jl + u - 1] : 0.0;
    double *pd = reinterpret_cast<double *>(pl);
    const int np = (n1 + 1) >> 1;
    for (int p0 = w * G; p0 < np; p0 += (NT / 64) * G) {
      const int p = p0 + g;
      const bool act = p < np;
      const bool hasb = act && 2 * p + 1 < n1;
      double *la = pd + (act ? 2 * p : 0);
      double *lb = la + 1;
      const double m1a = mu1[act ? 2 * p : 0];
      const double m1b = mu1[hasb ? 2 * p + 1 : 0];
      Cx<double> a[4], x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = half_in(la, lb, hasb, n1, jl + q * Q, N, act, sn[q]);
      wave_fft_line<double>(a, wb, lo, jl, lg0, twl, true);
      half_out(a, wb, lo, jl, lg0, cf, x);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 4 * jl + u;
        if (k >= 1) {
          const double sha = ab * ((m0[u] + m1a) + m2) + al;
          const double shb = ab * ((m0[u] + m1b) + m2) + al;
          const double sa = rsqrt(sha * sha + be * be);
          const double sb = rsqrt(shb * shb + be * be);
          if (act) {
            gacc += sa * (x[u].x * x[u].x);
            if (hasb) gacc += sb * (x[u].y * x[u].y);
          }
          x[u].x *= sa;
          x[u].y *= sb;
        } else {
          x[u] = Cx<double>{0.0, 0.0};
        }
      }
      // the scaled modes in natural order, then the inverse's input
      wave_lds_sync();
#pragma unroll
      for (int u = 0; u < 4; ++u) wb[lo + 4 * jl + u] = x[u];
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = half_in_buf(wb, lo, jl + q * Q, N, sn[q]);
      wave_fft_line<double>(a, wb, lo, jl, lg0, twl, true);
      half_out(a, wb, lo, jl, lg0, cf, x);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 4 * jl + u;
        if (act && k >= 1) {
          la[(k - 1) * n1] = x[u].x;
          if (hasb) lb[(k - 1) * n1] = x[u].y;
        }
      }
    }
  } else {
    const int L = 1 << lg0, Q = L >> 2, N = L >> 1;
    const int G = 64 >> (lg0 - 2);
    const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
    const int g = t >> (lg0 - 2), jl = t & (Q - 1);
    Cx<R> *wb = wbuf + w * kPlaneWaveElts;
    const int lo = g * L;
    const R ab = (R)S.abar_f, al = (R)S.alpha_f, be = (R)S.beta_f;
    const CSL_G R *mu0 = gbl(reinterpret_cast<const R *>(S.mu_f[0]));
    const CSL_G R *mu1 = gbl(reinterpret_cast<const R *>(S.mu_f[1]));
    const R m2 = gbl(reinterpret_cast<const R *>(S.mu_f[2]))[c];
    const R cf0 = (R)1 / sqrt((R)L);
    int md[4];
    R m0[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = jl + q * Q;
      md[q] = (k == 0 || k == N) ? -1 : (k < N ? k - 1 : L - 1 - k);
      m0[q] = md[q] >= 0 ? mu0[md[q]] : (R)0;
    }
    const int np = (n1 + 1) >> 1;
    for (int p0 = w * G; p0 < np; p0 += (NT / 64) * G) {
      const int p = p0 + g;
      const bool act = p < np;
      const bool hasb = act && 2 * p + 1 < n1;
      R *la = pl + (act ? 2 * p : 0);
      R *lb = la + 1;
      const R m1a = mu1[act ? 2 * p : 0];
      const R m1b = mu1[hasb ? 2 * p + 1 : 0];
      Cx<R> a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = pair_ext<R>(la, lb, hasb, n1, jl + q * Q, L, act);
      wave_fft_line<R>(a, wb, lo, jl, lg0, tw0, true);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Cx<R> v = dst_out(a[q], cf0);
        if (md[q] < 0) {
          v = Cx<R>{0, 0};
        } else {
          const R sha = ab * ((m0[q] + m1a) + m2) + al;
          const R shb = ab * ((m0[q] + m1b) + m2) + al;
          const R sa = (R)1 / sqrt(sha * sha + be * be);
          const R sb = (R)1 / sqrt(shb * shb + be * be);
          if (act && q < 2) {
            gacc += (double)sa * ((double)v.x * (double)v.x);
            if (hasb) gacc += (double)sb * ((double)v.y * (double)v.y);
          }
          v.x *= sa;
          v.y *= sb;
        }
        a[q] = v;
      }
      wave_fft_line<R>(a, wb, lo, jl, lg0, tw0, true);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = jl + q * Q;
        if (act && k >= 1 && k < N) {
          const Cx<R> v = dst_out(a[q], cf0);
          la[(k - 1) * n1] = v.x;
          if (hasb) lb[(k - 1) * n1] = v.y;
        }
      }
    }
  }
  __syncthreads();
  // axis 1 inverse, each wave storing its rows of T' once it has them
  CSL_G R *Tr = reinterpret_cast<CSL_G R *>(gbl(S.T)) + off;
  auto store = [&](int e0, int e1) {
    for (int e = e0 + lane; e < e1; e += 64) st_nt(Tr + e, pl[e]);
  };
  if constexpr (kHalf) plane_dst_pairs_half(pl, wbuf, tw1, n0, lg1, n1, 1, PlaneNoHook(), store);
  else plane_dst_pairs<R>(pl, wbuf, tw1, n0, lg1, n1, 1, PlaneNoHook(), store);
  const double sg = wg_sum(gacc, red);
  if (threadIdx.x == 0) S.part[tile] = sg;
}
#endif  // CSL_PLANE

template <int LDSB>
__device__ __forceinline__ void process_tile(const SysDesc &S, const IOPtr &io, int kind, int iter, int tile,
                             char *smem, double *red) {
#if CSL_2D_FFT_ONLY
  const bool d3 = false;
  const bool g = false;
#elif CSL_FFT_ONLY
  const bool d3 = (S.d == 3);
  const bool g = false;
#else
  const bool d3 = (S.d == 3);
  const int ax = (kind == K_X || kind == K_Z) ? S.d - 1 : (kind == K_Y ? 0 : 1);
  const bool g = S.gemm[ax] != 0;
#endif
  typedef FftEng<double, LDSB> F64;
  typedef FftEng<float, LDSB> F32;
  typedef GemmEng<double, LDSB> G64;
  typedef GemmEng<float, LDSB> G32;
#if CSL_GEMM16
  // FP16 split products: the preconditioner-precision passes of FP32
  // preconditioners on axes marked 2 (the FP64 row pass keeps G64)
  if (g && S.gemm[ax] == 2 && S.prec && kind != K_X && kind != K_PR) {
    typedef GemmEng16<LDSB> G16;
    if (kind == K_Z) {
      if (d3) tile_Z<float, 3, LDSB, G16>(S, io, iter, tile, smem);
      else tile_Z<float, 2, LDSB, G16>(S, io, iter, tile, smem);
    } else {
      if (d3) tile_Y<float, 3, LDSB, G16>(S, kind, iter, tile, smem, red);
      else tile_Y<float, 2, LDSB, G16>(S, kind, iter, tile, smem, red);
    }
    return;
  }
#endif
#if CSL_PLANE
  if (kind == K_X && S.plane && iter > 0 && S.lg[2] <= 8) {
    tile_XW<LDSB>(S, iter, tile, smem, red);
    return;
  }
  if (kind == K_Z && S.plane && S.lg[2] <= 8) {
#if CSL_PLANE_F64
    tile_ZW<double, LDSB>(S, io, iter, tile, smem);
#else
    tile_ZW<float, LDSB>(S, io, iter, tile, smem);
#endif
    return;
  }
  if (kind == K_Y && S.plane) {
    // one precision per instance (the runtime launches the one of S.prec)
#if CSL_PLANE_F64
    tile_YP<double>(S, iter, tile, smem, red);
#else
    tile_YP<float>(S, iter, tile, smem, red);
#endif
    return;
  }
#endif
  switch (kind) {
    case K_X:
      if (d3) g ? tile_X<3, LDSB, G64>(S, io, iter, tile, smem, red)
                : tile_X<3, LDSB, F64>(S, io, iter, tile, smem, red);
      else g ? tile_X<2, LDSB, G64>(S, io, iter, tile, smem, red)
             : tile_X<2, LDSB, F64>(S, io, iter, tile, smem, red);
      break;
    case K_Z:
      if (S.prec) {
        if (d3) g ? tile_Z<float, 3, LDSB, G32>(S, io, iter, tile, smem)
                  : tile_Z<float, 3, LDSB, F32>(S, io, iter, tile, smem);
        else g ? tile_Z<float, 2, LDSB, G32>(S, io, iter, tile, smem)
               : tile_Z<float, 2, LDSB, F32>(S, io, iter, tile, smem);
      } else {
        if (d3) g ? tile_Z<double, 3, LDSB, G64>(S, io, iter, tile, smem)
                  : tile_Z<double, 3, LDSB, F64>(S, io, iter, tile, smem);
        else g ? tile_Z<double, 2, LDSB, G64>(S, io, iter, tile, smem)
               : tile_Z<double, 2, LDSB, F64>(S, io, iter, tile, smem);
      }
      break;
    case K_PR:
      if (d3) tile_PR<3>(S, io, tile, red);
      else tile_PR<2>(S, io, tile, red);
      break;
    default:
      if (S.prec) {
        if (d3) g ? tile_Y<float, 3, LDSB, G32>(S, kind, iter, tile, smem, red)
                  : tile_Y<float, 3, LDSB, F32>(S, kind, iter, tile, smem, red);
        else g ? tile_Y<float, 2, LDSB, G32>(S, kind, iter, tile, smem, red)
               : tile_Y<float, 2, LDSB, F32>(S, kind, iter, tile, smem, red);
      } else {
        if (d3) g ? tile_Y<double, 3, LDSB, G64>(S, kind, iter, tile, smem, red)
                  : tile_Y<double, 3, LDSB, F64>(S, kind, iter, tile, smem, red);
        else g ? tile_Y<double, 2, LDSB, G64>(S, kind, iter, tile, smem, red)
               : tile_Y<double, 2, LDSB, F64>(S, kind, iter, tile, smem, red);
      }
      break;
  }
}

#if !CSL_SOLVE_ONLY
// ---------------------------------------------------------------------------
// Stand-alone P^{-1}: rows forward (x -> T), strided passes, rows inverse
// (T -> y), all in the preconditioner precision R.
// ---------------------------------------------------------------------------
template <typename R, int D, int LDSB, class E>
__device__ __forceinline__ void tile_pinv(const SysDesc &S, int pass, const double2 *x, double2 *y, int tile,
                          char *smem) {
  Cx<R> *buf = reinterpret_cast<Cx<R> *>(smem);
  // global views: the descriptor's generic pointer would compile to flat
  // accesses, which also count against the LDS wait counter
  CSL_G Cx<R> *T = gbl(reinterpret_cast<Cx<R> *>(S.T));
  const CSL_G double2 *X = gbl(x);
  CSL_G double2 *Y = gbl(y);
  // pass: 0 rows forward, 1 axis-1 forward, 2 axis-0 mid, 3 axis-1 inverse, 4 rows inverse
  const int ax = (pass == 0 || pass == 4) ? D - 1 : (pass == 2 ? 0 : 1);
  const int lp = (ax == D - 1) ? S.lpt_z : S.lpt_s[ax];
  const LineTile t = line_tile(S, ax, lp, tile);
  Cx<R> *twl = reinterpret_cast<Cx<R> *>(smem + LDSB);
  load_twiddles<R>(twl, t.lg);
  const R *Wm = E::matrix(S, ax);
  // T is column-blocked: the row passes reach it in blocked order, the
  // strided passes through their tile addressing
  if (pass == 0) E::template fill<4>(buf, t, [&](int, int, int p) { return to_cx<R>(ldg(X + p)); });
  else if (pass == 4) E::template fill_blk<4>(buf, t, [&](int, int, int q) { return ldg(T + q); });
  else E::template fill<4>(buf, t, [&](int, int, int p) { return ldg(T + p); });
  Cx<R> *o = E::transform(buf, t, twl, Wm);
  if (pass == 2) {
    const R ab = (sizeof(R) == 8) ? (R)S.abar : (R)S.abar_f;
    const R al = (sizeof(R) == 8) ? (R)S.alpha : (R)S.alpha_f;
    const R be = (sizeof(R) == 8) ? (R)S.beta : (R)S.beta_f;
    const CSL_G R *mu0;
    const CSL_G R *mu1;
    const CSL_G R *mu2;
    if constexpr (sizeof(R) == 8) {
      mu0 = gbl(reinterpret_cast<const R *>(S.mu[0]));
      mu1 = gbl(reinterpret_cast<const R *>(S.mu[1]));
      mu2 = gbl(reinterpret_cast<const R *>(S.mu[2]));
    } else {
      mu0 = gbl(reinterpret_cast<const R *>(S.mu_f[0]));
      mu1 = gbl(reinterpret_cast<const R *>(S.mu_f[1]));
      mu2 = gbl(reinterpret_cast<const R *>(S.mu_f[2]));
    }
    (void)E::scale_transform(buf, t, twl, Wm, [&](int l, int r) -> R {
      R lam;
      if (D == 2) {
        lam = mu0[r] + mu1[t.c0 + l];
      } else {
        lam = (mu0[r] + mu1[t.outer]) + mu2[t.c0 + l];
      }
      const R sh = ab * lam + al;
      return (R)1 / sqrt(sh * sh + be * be);
    }, &o);
  }
  // the next pass reads these in other workgroups: stream them past the L2
  if (pass == 4) {
    E::store(o, t, [&](int, int, int p, Cx<R> v) { st_nt(Y + p, (double)v.x, (double)v.y); });
  } else if (pass == 0) {
    E::store_blk(o, t, [&](int, int, int q, Cx<R> v) { st_nt(T + q, v); });
  } else {
    E::store(o, t, [&](int, int, int p, Cx<R> v) { st_nt(T + p, v); });
  }
}

#endif  // !CSL_SOLVE_ONLY

// ---------------------------------------------------------------------------
// Phase epilogue, run by the workgroup that completed the last tile of a
// phase: sums the tile partials in a fixed order, advances the Lanczos /
// Givens recurrences, takes the stopping decision and publishes the next
// phase of this system.
// ---------------------------------------------------------------------------
// The release exchange orders every earlier write of this thread (the reset
// completion count, the scalars) before the new ticket word; on gfx950 an
// agent-scope release writes back the L2, an acquire invalidates it, so no
// fence beyond the one the protocol needs is issued.
// Tiles of a phase that the workgroups of a single-system solve own from the
// start (sg = the grid size; 0 for a batch or while some workgroup of the grid
// has not started): each tile below min(sg, tiles) has one owner, which takes
// it the first time it sees the phase, without a claim, and the claim counter
// of the published phase starts after them.  Owners are used only once every
// workgroup is resident, so that progress never waits on one that is not.
__device__ __forceinline__ int static_tiles(const SysDesc &S, int kind, int sg) {
  return kind < K_NKINDS ? min(sg, S.ntile[kind]) : 0;
}

// Owned tile of workgroup b in a grid of g: workgroups are dealt to the 8
// XCDs round robin (b mod 8), and the workgroups of XCD x own tiles
// [start_x, start_x + count_x) in order, a bijection of [0, g).  The
// stencil's neighbouring rows then mostly come from tiles on the same XCD,
// whose L2 already holds them.
__device__ __forceinline__ int xcd_tile(int b, int g) {
  const int x = b & 7, i = b >> 3;
  const int q = g >> 3, r = g & 7;   // XCDs below r hold q + 1 workgroups
  return x * q + min(x, r) + i;
}

__device__ __forceinline__ void publish(const SysDesc &S, Ctl *C, int iter, int kind, int sg) {
  __hip_atomic_store(&C->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int s0 = static_tiles(S, kind, sg);
  const uint64_t w = make_word(iter, kind) + (s0 > 0 ? kWordOwned + (uint64_t)s0 : 0ull);
  __hip_atomic_exchange(&C->word, (unsigned long long)w, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void finish(const SysDesc &S, Glob *G, int iter, int status, int iters, double rt) {
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

// End a solve early at iteration iter with the iterate x_{iters}: if the
// update of step iter - 1 is still deferred, run one K_Z phase that applies
// it alone (ZM_FLUSH) and finish from its epilogue.
__device__ __forceinline__ void end_solve(const SysDesc &S, Glob *G, Ctl *C, int iter, int status,
                                          int iters, int sg) {
  if (C->pend) {
    C->pend = 0;
    C->zmode = ZM_FLUSH;
    C->fin_status = status;
    C->fin_iters = iters;
    publish(S, C, iter, K_Z, sg);
  } else {
    finish(S, G, iter, status, iters, __longlong_as_double(0x7ff8000000000000ll));
  }
}

__device__ __forceinline__ void epilogue(const SysDesc &S, const SolveParams &P, int kind, int iter, Glob *G,
                         double *red, int sg) {
  const int nt = S.ntile[kind];
  const bool last_strided = (kind == K_Y);   // carries the gamma^2 partials
  const bool need_sum = (kind == K_X) || (kind == K_PR) || last_strided;
  double a = 0.0;
  if (need_sum) {
    for (int i = threadIdx.x; i < nt; i += NT) a += S.part[i];
  }
  const double sum = need_sum ? wg_sum(a, red) : 0.0;
  if (threadIdx.x != 0) return;
  Ctl *C = S.ctl;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  // owners for the phases published here only once every workgroup has
  // started (recorded in the control block, so the count is read until then)
  if (sg > 0 && !C->owned_ok) {
    if (__hip_atomic_load(&G->arrived, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= sg)
      C->owned_ok = 1;
    else
      sg = 0;
  }
  const bool five = (S.d == 3) && !S.plane;   // 3-D with the three strided phases
  const int first_strided = five ? K_Y1 : K_Y;
  if (kind == K_X) {
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
        publish(S, C, 0, first_strided, sg);
      }
    } else if (!isfinite(sum)) {
      end_solve(S, G, C, iter, ST_NONFINITE, iter - 1, sg);
    } else {
      C->delta = sum;
      publish(S, C, iter, first_strided, sg);
    }
    return;
  }
  if (kind == K_Y1) {
    publish(S, C, iter, K_Y, sg);
    return;
  }
  if (kind == K_Y1I) {
    publish(S, C, iter, K_Z, sg);
    return;
  }
  if (last_strided) {
    const double g2 = sum;
    if (!isfinite(g2)) {
      S.info->relres_est = nan;
      if (iter == 0) finish(S, G, iter, ST_NONFINITE, 0, nan);
      else end_solve(S, G, C, iter, ST_NONFINITE, iter - 1, sg);
      return;
    }
    if (iter == 0) {
      if (g2 <= 0.0) {
        S.info->relres_est = nan;
        finish(S, G, iter, ST_BREAKDOWN, 0, nan);
        return;
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
      C->after_z = 0;
      C->pend = 0;
      publish(S, C, 0, five ? K_Y1I : K_Z, sg);
      return;
    }
    if (g2 < 0.0) {
      end_solve(S, G, C, iter, ST_BREAKDOWN, iter - 1, sg);
      return;
    }
    // Givens rotations of column j of the Lanczos tridiagonal (step j)
    const double gn = sqrt(g2);
    const double dl = C->delta, g = C->gamma;
    if (iter <= kLanczosCap) {
      S.lz[2 * (iter - 1)] = dl;
      S.lz[2 * (iter - 1) + 1] = gn;
      S.lz[2 * kLanczosCap] = (double)iter;
    }
    const double c = C->c, co = C->c_old, s = C->s, so = C->s_old, eta = C->eta;
    const double e0 = c * dl - co * s * g;
    const double e1 = hypot(e0, gn);
    const double e2 = s * dl + co * c * g;
    const double e3 = so * g;
    const double cn = e0 / e1, sn = gn / e1;
    if (C->pend) {
      // step j-1's update is still to be applied (with this step's)
      C->e1p = C->e1;
      C->e2p = C->e2;
      C->e3p = C->e3;
      C->cetap = C->ceta;
    }
    C->e1 = e1;
    C->e2 = e2;
    C->e3 = e3;
    C->ceta = cn * eta;
    C->eta = -sn * eta;
    C->c_old = c;
    C->c = cn;
    C->s_old = s;
    C->s = sn;
    C->gamma_old = g;
    C->gamma = gn;
    // decide what follows the update of x_j (phase K_Z)
    const double est = fabs(C->eta) / C->eta0;
    S.info->relres_est = est;
    if (gn == 0.0) {
      C->after_z = 2;
      C->finishing = ST_OK;
    } else if (est <= P.tol) {
      C->after_z = P.check_true ? 1 : 2;
      C->finishing = P.check_true ? -1 : ST_OK;
    } else if (iter >= P.maxit) {
      C->after_z = 2;
      C->finishing = ST_NOT_CONVERGED;
    } else {
      C->after_z = 0;
    }
    const int zm = C->pend ? ZM_PAIR : (C->after_z != 0 ? ZM_SINGLE : ZM_DEFER);
    C->zmode = zm;
    C->pend = (zm == ZM_DEFER);
    publish(S, C, iter, five ? K_Y1I : K_Z, sg);
    return;
  }
  if (kind == K_Z) {
    if (iter > 0 && C->zmode == ZM_FLUSH) finish(S, G, iter, C->fin_status, C->fin_iters, nan);
    else if (iter == 0 || C->after_z == 0) publish(S, C, iter + 1, K_X, sg);
    else publish(S, C, iter, K_PR, sg);
    return;
  }
  if (kind == K_PR) {
    const int k = iter;
    const double rt = sqrt(sum) / C->bnorm;
    if (C->finishing >= 0) {
      finish(S, G, iter, C->finishing, k, rt);
    } else if (rt <= P.tol) {
      finish(S, G, iter, ST_OK, k, rt);
    } else if (k >= P.maxit) {
      finish(S, G, iter, ST_NOT_CONVERGED, k, rt);
    } else {
      publish(S, C, iter + 1, K_X, sg);
    }
    return;
  }
}

// ---------------------------------------------------------------------------
// Persistent solver: every workgroup repeatedly claims a tile of whichever
// system has one ready, processes it, and the workgroup that completes a
// phase runs its epilogue.  A workgroup never waits while holding a tile,
// so progress does not depend on which workgroups are resident.  Idle
// workgroups exit when every system is done or the time limit passes; past
// the limit no phase is published any more, so a system stops where it is
// (status left unset) instead of running on in the workgroups still busy.
// ---------------------------------------------------------------------------
template <int LDSB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(CSL_WAVES_PER_EU))) void solve_kernel(
    const SysDesc *__restrict__ sys, const IOPtr *__restrict__ io, IOPtr io0, int nsys,
    SolveParams P, Glob *G) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[NT / 64];
  __shared__ int sh_s, sh_tile, sh_kind, sh_iter, sh_last;
  const int tid = threadIdx.x;
  twiddle_cache_reset();
  int cur = blockIdx.x % nsys;
  const long long t0 = wall_clock64();
  int backoff = 0;
  // Longest back-off, in rounds of s_sleep(8): a single system leaves every
  // workgroup idle between its phases, and one round (about 0.2 us) takes up
  // the next phase soonest; a batch keeps workgroups busy with other
  // systems, and polls less (about 14 us).
  const int bcap = nsys > 1 ? 64 : 1;
  // a single system: once every workgroup has started, phases are published
  // with tiles 0 .. min(grid, tiles) - 1 owned by workgroups, one each
  // (xcd_tile)
  const int sg = nsys == 1 ? (int)gridDim.x : 0;
  if (tid == 0) __hip_atomic_fetch_add(&G->arrived, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned seen = 0xffffffffu;   // [iter | kind] of the last owned tile taken
  for (;;) {
    if (tid < 64) {
      const int lane = tid;
      int found = -1;
      if (sg > 0) {
        // single system: the workgroup's own tile of a phase it has not
        // served yet, else a tile past the owned ones from the counter
        if (lane == 0) {
          const uint64_t w = __hip_atomic_load(&sys[0].ctl->word, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
          const int kd = word_kind(w);
          if (kd < K_NKINDS) {
            const int it = word_iter(w);
            const unsigned key = (unsigned)(w >> 32);
            // workgroup b (on XCD b mod 8) owns tile xcd_tile(b): each XCD a
            // contiguous run of tiles, so neighbouring tiles share an L2
            const int own = xcd_tile((int)blockIdx.x, sg);
            if (word_owned(w) && key != seen && own < static_tiles(sys[0], kd, sg)) {
              seen = key;
              sh_tile = own;
              sh_kind = kd;
              sh_iter = it;
              found = 0;
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            } else if (word_next(w) < (uint32_t)sys[0].ntile[kd]) {
              const uint64_t w2 = __hip_atomic_fetch_add(&sys[0].ctl->word, 1ull, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
              const int kd2 = word_kind(w2);
              if (kd2 < K_NKINDS && word_next(w2) < (uint32_t)sys[0].ntile[kd2]) {
                sh_tile = (int)word_next(w2);
                sh_kind = kd2;
                sh_iter = word_iter(w2);
                found = 0;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
              }
            }
          }
        }
        found = __shfl(found, 0, 64);
      }
      // Otherwise wave 0 looks at up to 64 systems per round trip: each lane
      // loads one ticket word, a ballot lists the systems with a tile ready,
      // and lanes try to claim one in order, starting from the last system
      // served.
      for (int base = 0; sg == 0 && base < nsys && found == -1; base += 64) {
        const int k = base + lane;
        int sl = cur + k;
        while (sl >= nsys) sl -= nsys;
        bool avail = false;
        if (k < nsys) {
          const uint64_t w = __hip_atomic_load(&sys[sl].ctl->word, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
          const int kd = word_kind(w);
          avail = kd < K_NKINDS && word_next(w) < (uint32_t)sys[sl].ntile[kd];
        }
        unsigned long long mask = __ballot(avail);
        while (mask != 0ull && found == -1) {
          const int ln = __ffsll((long long)mask) - 1;
          mask &= mask - 1ull;
          int got = 0;
          if (lane == ln) {
            // relaxed claim; the acquire fence below, taken only when a tile
            // was obtained, synchronises with the release that published the
            // phase (an acquiring increment would invalidate the L2 on every
            // attempt, a second time on success)
            const uint64_t w2 = __hip_atomic_fetch_add(&sys[sl].ctl->word, 1ull,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int kd2 = word_kind(w2);
            if (kd2 < K_NKINDS && word_next(w2) < (uint32_t)sys[sl].ntile[kd2]) {
              got = 1;
              sh_tile = (int)word_next(w2);
              sh_kind = kd2;
              sh_iter = word_iter(w2);
              // make the previous phase's results visible to this workgroup
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
          }
          got = __shfl(got, ln, 64);
          if (got) found = __shfl(sl, ln, 64);
        }
      }
      if (found >= 0) {
        cur = found;
        backoff = 0;
      } else {
        // nothing ready: stop when every system is done or on error / time
        // limit, else back off exponentially (up to bcap rounds) before looking again
        if (__hip_atomic_load(&G->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0 ||
            __hip_atomic_load(&G->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          found = -2;
        } else if (wall_clock64() - t0 > P.timeout_ticks) {
          if (lane == 0)
            __hip_atomic_fetch_or(&G->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          found = -2;
        } else {
          backoff = backoff < bcap ? backoff * 2 + 1 : bcap;
          for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(8);
        }
      }
      if (lane == 0) sh_s = found;
    }
    __syncthreads();
    const int s = sh_s;
    if (s == -2) break;
    if (s >= 0) {
      const int kind = sh_kind, iter = sh_iter, tile = sh_tile;
      const SysDesc &S = sys[s];
      const IOPtr iop = io ? io[s] : io0;
      process_tile<LDSB>(S, iop, kind, iter, tile, smem, red);
      // every wave's stores are complete at the barrier; one agent-scope
      // release fence then publishes them with the (relaxed) completion
      // count, and only the workgroup that completes the phase acquires
      __syncthreads();
      if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned old = __hip_atomic_fetch_add(&S.ctl->done, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        int last = (old + 1 == (unsigned)S.ntile[kind]);
        if (last) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          // past the time limit the next phase is not published: every
          // system stops within one phase and the idle workgroups exit
          if (wall_clock64() - t0 > P.timeout_ticks) {
            __hip_atomic_fetch_or(&G->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = 0;
          }
        }
        sh_last = last;
      }
      __syncthreads();
      if (sh_last) epilogue(S, P, kind, iter, G, red, sg);
    }
    __syncthreads();
  }
}

#if !CSL_SOLVE_ONLY
__global__ void init_kernel(const SysDesc *__restrict__ sys, int nsys, Glob *G) {
  for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
    Ctl *C = sys[s].ctl;
    C->word = make_word(0, K_X);
    C->done = 0;
    C->finishing = -1;
    C->after_z = 0;
    C->pend = 0;
    C->zmode = ZM_DEFER;
    C->owned_ok = 0;
    DevInfo *I = sys[s].info;
    I->status = -1;
    I->iters = 0;
    I->relres_est = 0.0;
    I->relres_true = 0.0;
    sys[s].lz[2 * kLanczosCap] = 0.0;
  }
  if (threadIdx.x == 0) {
    G->active = nsys;
    G->error = 0;
    G->arrived = 0;
  }
}

// Descriptor of a system whose workspaces the caller placed in a buffer of
// its own: the descriptor arrives by value and is stored at dst, and the
// per-axis eigenvalue tables mu_k = (4 / h^2) sin^2(k pi / (2 (n + 1))) of L
// it points to are filled in FP64 and FP32 (0 on the axes past the grid's
// dimension).  One workgroup.
__global__ void write_desc_kernel(SysDesc h, SysDesc *dst) {
  if (threadIdx.x == 0) *dst = h;
  for (int ax = 0; ax < 3; ++ax) {
    double *mu = const_cast<double *>(h.mu[ax]);
    float *muf = const_cast<float *>(h.mu_f[ax]);
    const int n = h.n[ax];
    for (int k = 1 + (int)threadIdx.x; k <= n; k += blockDim.x) {
      const double sv = sin((double)k * M_PI / (2.0 * (n + 1)));
      const double m = ax < h.d ? 4.0 * h.h2[ax] * sv * sv : 0.0;
      mu[k - 1] = m;
      muf[k - 1] = (float)m;
    }
  }
}

// ---------------------------------------------------------------------------
// Stand-alone operators.
// ---------------------------------------------------------------------------
// y = A x on a 3-D grid, marching.  Every wave owns a strip of up to 64
// points along the contiguous axis (i2) at one i1 and walks a slab of
// planes along axis 0, keeping x and a of the planes i0 - 1, i0, i0 + 1 in
// registers: each value comes from HBM once, as the next plane, the face
// coefficient between two planes is formed once and carried to the next
// step, and the neighbours and faces along i2 come from the adjacent lanes.
// The arithmetic is that of stencil_apply: the same face expressions, then
// the sum over the axes in order.
// Strips are numbered slab-major, then i1, then the i2 block, and each XCD
// (workgroup b runs on XCD b mod 8) takes one eighth of that order, so the
// strips at i1 +- 1 that a strip reads sit in the same L2.
__device__ __forceinline__ double harm_face(double lo, double hi, double h2) {
  return (2.0 * lo * hi / (lo + hi)) * h2;
}

__device__ __forceinline__ double2 shfl2(double2 v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

__global__ __launch_bounds__(NT) void apply_A_march3_kernel(const SysDesc *__restrict__ sys,
                                                            const double2 *__restrict__ x,
                                                            double2 *__restrict__ y, int nslab) {
  const SysDesc &S = *sys;
  const int n0 = S.n[0], n1 = S.n[1], n2 = S.n[2];
  const int st0 = S.st[0], st1 = S.st[1];
  const int lane = threadIdx.x & 63;
  const int xb = (n2 + 63) >> 6;            // strips per line along i2
  const int per_slab = n1 * xb;
  const int total = nslab * per_slab;
  // wave -> strip: XCD k walks strips [k total / 8, (k + 1) total / 8)
  const int nxcd = 8;
  const int xcd = blockIdx.x % nxcd, wg = blockIdx.x / nxcd;
  const int w = wg * (NT / 64) + ((int)threadIdx.x >> 6);
  const int lo_s = (int)((long long)total * xcd / nxcd);
  const int hi_s = (int)((long long)total * (xcd + 1) / nxcd);
  const int strip = lo_s + w;
  if (strip >= hi_s) return;                // whole waves leave together
  const int slab = strip / per_slab;
  const int rem = strip - slab * per_slab;
  const int i1 = rem / xb;
  const int i2 = (rem - i1 * xb) * 64 + lane;
  const bool valid = i2 < n2;
  const int s0 = (int)((long long)n0 * slab / nslab);
  const int s1 = (int)((long long)n0 * (slab + 1) / nslab);
  const CSL_G double2 *__restrict__ xg = gbl(x);
  const CSL_G double *__restrict__ A = gbl(S.a);
  CSL_G double2 *__restrict__ yg = gbl(y);
  const double h0 = S.h2[0], h1 = S.h2[1], h2 = S.h2[2];
  const double al = S.alpha, be = S.beta;
  const double2 zero = make_double2(0.0, 0.0);
  const bool lo1 = i1 > 0, hi1 = i1 < n1 - 1;
  const bool lo2 = valid && i2 > 0, hi2 = valid && i2 < n2 - 1;
  const int q = i1 * st1 + (valid ? i2 : 0);
  int p = s0 * st0 + q;
  double2 xc = valid ? ldg(xg + p) : zero;
  double ac = valid ? A[p] : 1.0;
  double2 xm = zero;
  double fb0;
  if (s0 > 0) {
    xm = valid ? ldg(xg + (p - st0)) : zero;
    const double am = valid ? A[p - st0] : 1.0;
    fb0 = harm_face(am, ac, h0);
  } else {
    fb0 = ac * h0;
  }
  for (int i0 = s0; i0 < s1; ++i0, p += st0) {
    const bool up0 = i0 < n0 - 1;
    const double2 xp = (valid && up0) ? ldg(xg + (p + st0)) : zero;
    const double ap = (valid && up0) ? A[p + st0] : 1.0;
    // axis 1: the strips at i1 +- 1
    const double2 xb1 = (valid && lo1) ? ldg(xg + (p - st1)) : zero;
    const double2 xa1 = (valid && hi1) ? ldg(xg + (p + st1)) : zero;
    const double ab1 = (valid && lo1) ? A[p - st1] : 1.0;
    const double aa1 = (valid && hi1) ? A[p + st1] : 1.0;
    // axis 2: neighbours from the adjacent lanes, the strip ends from memory
    double2 xb2 = shfl2(xc, lane > 0 ? lane - 1 : 0);
    double ab2 = __shfl(ac, lane > 0 ? lane - 1 : 0, 64);
    if (lane == 0 && lo2) {
      xb2 = ldg(xg + (p - 1));
      ab2 = A[p - 1];
    }
    double2 xa2 = shfl2(xc, lane < 63 ? lane + 1 : 63);
    if (lane == 63 && hi2) xa2 = ldg(xg + (p + 1));
    // faces: axis 0 below is carried, above formed now; axis 2 above is the
    // lower face of the next lane
    const double fa0 = up0 ? harm_face(ac, ap, h0) : ac * h0;
    const double fb1 = lo1 ? harm_face(ab1, ac, h1) : ac * h1;
    const double fa1 = hi1 ? harm_face(ac, aa1, h1) : ac * h1;
    const double fb2 = lo2 ? harm_face(ab2, ac, h2) : ac * h2;
    double fa2 = __shfl(fb2, lane < 63 ? lane + 1 : 63, 64);
    if (lane == 63 && hi2) fa2 = harm_face(ac, A[p + 1], h2);
    if (!hi2) fa2 = ac * h2;
    const double2 cb0 = (i0 > 0) ? xm : zero;
    const double2 ca0 = xp;
    const double2 cb2 = lo2 ? xb2 : zero;
    const double2 ca2 = hi2 ? xa2 : zero;
    double rx = 0.0, ry = 0.0;
    rx += fb0 * (xc.x - cb0.x) + fa0 * (xc.x - ca0.x);
    ry += fb0 * (xc.y - cb0.y) + fa0 * (xc.y - ca0.y);
    rx += fb1 * (xc.x - xb1.x) + fa1 * (xc.x - xa1.x);
    ry += fb1 * (xc.y - xb1.y) + fa1 * (xc.y - xa1.y);
    rx += fb2 * (xc.x - cb2.x) + fa2 * (xc.x - ca2.x);
    ry += fb2 * (xc.y - cb2.y) + fa2 * (xc.y - ca2.y);
    // y = (K + lambda I) conj(x) = conj(K x + conj(lambda) x)
    const double ux = rx + al * xc.x + be * xc.y;
    const double uy = ry + al * xc.y - be * xc.x;
    if (valid) st_nt(yg + p, ux, -uy);
    xm = xc;
    xc = xp;
    ac = ap;
    fb0 = fa0;
  }
}

// y = A x over the whole grid.  The points are split into 8 contiguous
// slabs, one per XCD (workgroup b runs on XCD b mod 8), and the workgroups
// of one XCD sweep their slab in steps of NT points, so the neighbouring
// rows and planes a point needs were read moments before into the same L2:
// x and a come from HBM about once, y goes back once (the model's 40 bytes
// per point).
template <int D>
__global__ __launch_bounds__(NT) void apply_A_kernel(const SysDesc *__restrict__ sys,
                                                     const double2 *__restrict__ x,
                                                     double2 *__restrict__ y) {
  const SysDesc &S = *sys;
  const int nlast = S.n[D - 1];
  const int nxcd = 8;
  const int slab = blockIdx.x % nxcd, w = blockIdx.x / nxcd, nw = gridDim.x / nxcd;
  const int p0 = (int)((long long)S.M * slab / nxcd);
  const int p1 = (int)((long long)S.M * (slab + 1) / nxcd);
  const CSL_G double2 *__restrict__ xg = gbl(x);
  CSL_G double2 *__restrict__ yg = gbl(y);
  const double al = S.alpha, be = S.beta;
  for (int p = p0 + w * NT + (int)threadIdx.x; p < p1; p += nw * NT) {
    const int row = p / nlast;
    int idx[3];
    row_index<D>(S, row, p - row * nlast, idx);
    const StencilIn<D> in = stencil_load<D>(S, xg, p, idx);
    const double2 kx = stencil_apply<D>(S, in);
    const double2 xv = in.c;
    // y = (K + lambda I) conj(x) = conj(K x + conj(lambda) x)
    const double ux = kx.x + al * xv.x + be * xv.y;
    const double uy = kx.y + al * xv.y - be * xv.x;
    st_nt(yg + p, ux, -uy);
  }
}

template <typename R, int D, int LDSB>
__global__ __launch_bounds__(NT) void pinv_pass_kernel(const SysDesc *__restrict__ sys, int pass,
                                                       const double2 *x, double2 *y) {
  extern __shared__ __align__(16) char smem[];
  const SysDesc &S = *sys;
  const int ax = (pass == 0 || pass == 4) ? D - 1 : (pass == 2 ? 0 : 1);
  if constexpr (sizeof(R) == 4) {
    if (S.gemm[ax] == 2) {
      tile_pinv<R, D, LDSB, GemmEng16<LDSB>>(S, pass, x, y, blockIdx.x, smem);
      return;
    }
  }
  if (S.gemm[ax]) tile_pinv<R, D, LDSB, GemmEng<R, LDSB>>(S, pass, x, y, blockIdx.x, smem);
  else tile_pinv<R, D, LDSB, FftEng<R, LDSB>>(S, pass, x, y, blockIdx.x, smem);
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
// Transform over the L = 2^lg steps of an all-at-once vector (L vectors of M
// complex values, step-major) that block-diagonalises the alpha-circulant
// time factor:
//   forward: y_j = sum_k exp(-2 pi i j k / L) alpha^(k/L) x_k
//   inverse: y_k = alpha^(-k/L) / L sum_j exp(2 pi i j k / L) x_j
// (the inverse as the conjugate of the forward DFT of the conjugate).  A
// workgroup takes P = MAXE / L consecutive grid points, reads their L values
// step by step (P consecutive points per step: coalesced), transforms the P
// lines of length L in LDS and writes them back the same way.  ln_alpha_l is
// ln(alpha) / L.
// ---------------------------------------------------------------------------
template <int LDSB>
__global__ __launch_bounds__(NT) void step_transform_kernel(const double2 *__restrict__ x,
                                                            double2 *__restrict__ y, int M,
                                                            int lg, double ln_alpha_l,
                                                            int inverse) {
  extern __shared__ __align__(16) char smem[];
  constexpr int MAXE = MaxElts<double, LDSB>::value;
  Cx<double> *buf = reinterpret_cast<Cx<double> *>(smem);
  Cx<double> *twl = reinterpret_cast<Cx<double> *>(smem + LDSB);
  const int L = 1 << lg;
  const int lgp = ilog2i(MAXE) - lg;   // log2 of the points per workgroup
  const int P = 1 << lgp;
  // block of points by XCD (xcd_tile): a step's run of P points rarely starts
  // on a 128-byte line (M is odd), so neighbouring blocks share a line at
  // every step; dealt by XCD, the two blocks run on one XCD one after the
  // other, the shared line is fetched once into its L2, and the outputs use
  // plain (write-back) stores, so that the two halves of a shared line meet
  // in that L2 and leave it as one line
  const long long p0 = (long long)xcd_tile((int)blockIdx.x, (int)gridDim.x) * P;
  const CSL_G double2 *__restrict__ X = gbl(x);
  CSL_G double2 *__restrict__ Y = gbl(y);
  load_twiddles<double>(twl, lg);
  // L P = MAXE: every thread moves MAXE / NT values each way; all loads are
  // issued before the first LDS write
  constexpr int U = MAXE / NT;
  double2 u[U];
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int e = threadIdx.x + i * NT;
    const long long p = p0 + (e & (P - 1));
    u[i] = p < M ? ldg(X + (long long)(e >> lgp) * M + p) : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int e = threadIdx.x + i * NT;
    const int k = e >> lgp, pl = e & (P - 1);
    Cx<double> v;
    if (inverse) {
      v = {u[i].x, -u[i].y};
    } else {
      const double g = exp(ln_alpha_l * k);
      v = {u[i].x * g, u[i].y * g};
    }
    buf[pl * L + k] = v;
  }
  __syncthreads();
  fft_lines<double, LDSB>(buf, P, lg, twl);
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int e = threadIdx.x + i * NT;
    const int k = e >> lgp, pl = e & (P - 1);
    const long long p = p0 + pl;
    if (p < M) {
      const Cx<double> v = buf[pl * L + k];
      if (inverse) {
        const double g = exp(-ln_alpha_l * k) / L;
        *(CSL_G nt_d2 *)(Y + (long long)k * M + p) = nt_d2{v.x * g, -v.y * g};
      } else {
        *(CSL_G nt_d2 *)(Y + (long long)k * M + p) = nt_d2{v.x, v.y};
      }
    }
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

#endif  // !CSL_SOLVE_ONLY

// ---------------------------------------------------------------------------
// Host-side launch wrappers (declared in csl_kernels.hpp).
// ---------------------------------------------------------------------------
hipError_t upload_twiddles(const double2 *tw64, const float2 *tw32) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_tw64), tw64, sizeof(double2) * TWN);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tw32), tw32, sizeof(float2) * TWN);
}

hipError_t launch_solve(const SysDesc *dsys, const IOPtr *dio, IOPtr io0, int nsys,
                        const SolveParams &P, Glob *G, int grid, size_t smem, hipStream_t s) {
#if CSL_PLANE
  // the plane phase uses the whole LDS (the row phases its first 72 KiB)
  (void)smem;
  hipLaunchKernelGGL(solve_kernel<65536>, dim3(grid), dim3(NT), kPlaneLdsBytes, s, dsys, dio, io0,
                     nsys, P, G);
#else
  if (smem <= 32768)
    hipLaunchKernelGGL(solve_kernel<32768>, dim3(grid), dim3(NT), 32768 + tw_lds_bytes(32768), s, dsys, dio,
                       io0, nsys, P, G);
  else
    hipLaunchKernelGGL(solve_kernel<65536>, dim3(grid), dim3(NT), 65536 + tw_lds_bytes(65536), s, dsys, dio,
                       io0, nsys, P, G);
#endif
  return hipGetLastError();
}

hipError_t solve_occupancy(size_t smem, int *blocks_per_cu) {
#if CSL_PLANE
  (void)smem;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, solve_kernel<65536>, NT,
                                                      kPlaneLdsBytes);
#else
  if (smem <= 32768)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, solve_kernel<32768>, NT,
                                                        32768 + tw_lds_bytes(32768));
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, solve_kernel<65536>, NT,
                                                      65536 + tw_lds_bytes(65536));
#endif
}

#if !CSL_SOLVE_ONLY
hipError_t launch_init(const SysDesc *dsys, int nsys, Glob *G, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(64), 0, s, dsys, nsys, G);
  return hipGetLastError();
}

hipError_t launch_write_desc(const SysDesc &h, SysDesc *dst, hipStream_t s) {
  hipLaunchKernelGGL(write_desc_kernel, dim3(1), dim3(256), 0, s, h, dst);
  return hipGetLastError();
}

// 3-D grids with at least 16 planes march (about 16K waves, slabs of at least
// 8 planes); other grids use the point-wise kernel.
static hipError_t launch_apply_A3(const SysDesc *dsys, const int n[3], const double2 *x,
                                  double2 *y, hipStream_t s) {
  const int xb = (n[2] + 63) / 64;
  const int per_slab = n[1] * xb;
  int nslab = 16384 / (per_slab > 0 ? per_slab : 1);
  const int maxslab = n[0] / 8 > 0 ? n[0] / 8 : 1;
  nslab = nslab < 1 ? 1 : (nslab > maxslab ? maxslab : nslab);
  const int waves = nslab * per_slab;
  const int per_xcd_waves = (waves + 7) / 8;
  const int wgs_per_xcd = (per_xcd_waves + NT / 64 - 1) / (NT / 64);
  hipLaunchKernelGGL(apply_A_march3_kernel, dim3(8 * wgs_per_xcd), dim3(NT), 0, s, dsys, x, y,
                     nslab);
  return hipGetLastError();
}

hipError_t launch_apply_A(const SysDesc *dsys, int d, const int n[3], int M, const double2 *x,
                          double2 *y, hipStream_t s) {
  if (d == 3 && n[0] >= 16) return launch_apply_A3(dsys, n, x, y, s);
  // 8 slabs (one per XCD), up to 256 workgroups sweeping each
  const int per = (M / 8 + NT - 1) / NT;
  const int grid = 8 * (per < 1 ? 1 : (per > 256 ? 256 : per));
  if (d == 3) hipLaunchKernelGGL(apply_A_kernel<3>, dim3(grid), dim3(NT), 0, s, dsys, x, y);
  else hipLaunchKernelGGL(apply_A_kernel<2>, dim3(grid), dim3(NT), 0, s, dsys, x, y);
  return hipGetLastError();
}

template <int LDSB>
static void pinv_launch(const SysDesc *dsys, int d, int prec, int pass, int ntile, size_t smem,
                        const double2 *x, double2 *y, hipStream_t s) {
  if (prec) {
    if (d == 3)
      hipLaunchKernelGGL((pinv_pass_kernel<float, 3, LDSB>), dim3(ntile), dim3(NT), smem, s, dsys, pass, x, y);
    else
      hipLaunchKernelGGL((pinv_pass_kernel<float, 2, LDSB>), dim3(ntile), dim3(NT), smem, s, dsys, pass, x, y);
  } else {
    if (d == 3)
      hipLaunchKernelGGL((pinv_pass_kernel<double, 3, LDSB>), dim3(ntile), dim3(NT), smem, s, dsys, pass, x, y);
    else
      hipLaunchKernelGGL((pinv_pass_kernel<double, 2, LDSB>), dim3(ntile), dim3(NT), smem, s, dsys, pass, x, y);
  }
}

hipError_t launch_pinv_pass(const SysDesc *dsys, int d, int prec, int pass, int ntile, size_t smem,
                            const double2 *x, double2 *y, hipStream_t s) {
  if (smem <= 32768) pinv_launch<32768>(dsys, d, prec, pass, ntile, 32768 + tw_lds_bytes(32768), x, y, s);
  else pinv_launch<65536>(dsys, d, prec, pass, ntile, 65536 + tw_lds_bytes(65536), x, y, s);
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

hipError_t launch_step_transform(const double2 *x, double2 *y, int M, int lg, double alpha_c,
                                 int inverse, hipStream_t s) {
  constexpr int LDSB = 32768;
  const int P = MaxElts<double, LDSB>::value >> lg;
  const long long nblk = ((long long)M + P - 1) / P;
  hipLaunchKernelGGL(step_transform_kernel<LDSB>, dim3((unsigned)nblk), dim3(NT),
                     LDSB + tw_lds_bytes(LDSB), s, x, y, M, lg, log(alpha_c) / (1 << lg),
                     inverse);
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

#endif  // !CSL_SOLVE_ONLY

}  // namespace CSL_KNS
}  // namespace csl
