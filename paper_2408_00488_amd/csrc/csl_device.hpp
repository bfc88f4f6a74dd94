// Device building blocks for gfx950: complex helpers, LDS-staged sine
// transforms (DST-I through a radix-4/2 Stockham FFT of the odd extension),
// the variable-coefficient stencil, and the phase tiles of the MINRES
// iteration.  Everything here runs inside workgroups of NT threads.
//
// The device code is compiled once per workgroup size: CSL_NT threads, in
// namespace csl::CSL_KNS (256 threads in csl::wg256 unless the including
// file says otherwise), so that each instance has its own kernels, twiddle
// tables and register allocation.
#pragma once
#include "csl_common.hpp"

#ifndef CSL_NT
#define CSL_NT 256
#endif
#ifndef CSL_KNS
#define CSL_KNS wg256
#endif

// Elements per thread and round of the pipelined fills and stores, scaled
// with the block size so that a workgroup keeps the same number of loads in
// flight (and a thread the same registers per element) at either size.
#define CSL_U(u) ((u) * 256 / CSL_NT > 0 ? (u) * 256 / CSL_NT : 1)

namespace csl {
namespace CSL_KNS {

constexpr int NT = CSL_NT;   // threads per workgroup (NT / 64 wave64)

template <typename R>
struct alignas(2 * sizeof(R)) Cx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ Cx<R> csub(Cx<R> a, Cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Twiddle tables exp(-2 pi i m / TWN), m < TWN, filled by the host runtime.
__device__ double2 g_tw64[TWN];
__device__ float2 g_tw32[TWN];

template <typename R> __device__ __forceinline__ const Cx<R> *twiddles();
template <> __device__ __forceinline__ const Cx<double> *twiddles<double>() {
  return reinterpret_cast<const Cx<double> *>(g_tw64);
}
template <> __device__ __forceinline__ const Cx<float> *twiddles<float>() {
  return reinterpret_cast<const Cx<float> *>(g_tw32);
}

// Global-memory views of the pointers held in the descriptors.  Accesses
// through an address-space-1 pointer compile to global_* instructions
// instead of flat_* ones; flat accesses also count against the LDS wait
// counter, so every LDS wait would otherwise stall on outstanding HBM loads
// and stores.
#define CSL_G __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ CSL_G T *gbl(T *p) {
  return (CSL_G T *)p;
}
template <typename T>
__device__ __forceinline__ const CSL_G T *gbl(const T *p) {
  return (const CSL_G T *)p;
}

typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));

// Loads through the global views (the vector classes cannot be copied out of
// another address space, the builtin vector types can).
__device__ __forceinline__ double2 ldg(const CSL_G double2 *p) {
  const nt_d2 v = *(const CSL_G nt_d2 *)p;
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ Cx<double> ldg(const CSL_G Cx<double> *p) {
  const nt_d2 v = *(const CSL_G nt_d2 *)p;
  return Cx<double>{v.x, v.y};
}
__device__ __forceinline__ Cx<float> ldg(const CSL_G Cx<float> *p) {
  const nt_f2 v = *(const CSL_G nt_f2 *)p;
  return Cx<float>{v.x, v.y};
}

// Streaming stores for vectors that the next phase reads from other
// workgroups: the nontemporal hint keeps them from lingering dirty in L2,
// which both speeds up the stream and shortens the L2 write-back that every
// tile's release performs.
__device__ __forceinline__ void st_nt(CSL_G double2 *p, double x, double y) {
  const nt_d2 v = {x, y};
  __builtin_nontemporal_store(v, (CSL_G nt_d2 *)p);
}
__device__ __forceinline__ void st_nt(CSL_G double *p, double v) {
  __builtin_nontemporal_store(v, p);
}
__device__ __forceinline__ void st_nt(CSL_G float *p, float v) {
  __builtin_nontemporal_store(v, p);
}
__device__ __forceinline__ void st_nt(CSL_G Cx<double> *p, Cx<double> c) {
  const nt_d2 v = {c.x, c.y};
  __builtin_nontemporal_store(v, (CSL_G nt_d2 *)p);
}
__device__ __forceinline__ void st_nt(CSL_G Cx<float> *p, Cx<float> c) {
  const nt_f2 v = {c.x, c.y};
  __builtin_nontemporal_store(v, (CSL_G nt_f2 *)p);
}

// Elements of the LDS line buffer for an LDS budget of LDSB bytes.
template <typename R, int LDSB> struct MaxElts {
  static constexpr int value = LDSB / (int)sizeof(Cx<R>);
};

// ---------------------------------------------------------------------------
// In-LDS complex FFT of `nl` lines of length L = 2^lg stored back to back.
// Stockham autosort: a radix-2 stage first when lg is odd, then radix-4
// stages; each stage reads all of its inputs into registers, synchronises,
// and writes the outputs in place.  Output is in natural order.
// ---------------------------------------------------------------------------
// LDS bytes reserved after a line buffer of LDSB bytes for the twiddles of
// one length: L/4 entries, L <= 1024 with a 32 KiB buffer, L <= 2048 else.
constexpr int tw_lds_bytes(int ldsb) { return ldsb <= 32768 ? 4096 : 8192; }

// Stage exp(-2 pi i m / L), m < L/4, into LDS: every radix-4 stage of a
// length-L Stockham FFT uses w1 = exp(-2 pi i k / (4 Ns)), k < Ns, which is
// entry k L / (4 Ns) < L/4 of that table.
template <typename R>
__device__ __forceinline__ void load_twiddles(Cx<R> *twl, int lg) {
  const Cx<R> *tw = twiddles<R>();
  const int q = (1 << lg) >> 2;
  const int step = TWN >> lg;
  for (int m = threadIdx.x; m < q; m += NT) twl[m] = tw[m * step];
  __syncthreads();
}

// Persistent workgroups keep the staged table between tiles: the key (length
// and precision of the table in LDS) is reset at kernel start and the table
// is reloaded only when a tile needs another one.
__shared__ int s_twkey;

__device__ __forceinline__ void twiddle_cache_reset() {
  if (threadIdx.x == 0) s_twkey = -1;
}

template <typename R>
__device__ __forceinline__ void load_twiddles_cached(Cx<R> *twl, int lg) {
  const int key = lg * 2 + (sizeof(R) == 4 ? 1 : 0);
  if (s_twkey == key) return;   // uniform: every thread reads the same LDS word
  load_twiddles<R>(twl, lg);
  if (threadIdx.x == 0) s_twkey = key;
}

template <typename R, int LDSB>
__device__ __forceinline__ void fft_lines(Cx<R> *buf, int nl, int lg, const Cx<R> *twl) {
  constexpr int MAXE = MaxElts<R, LDSB>::value;
  const int tid = threadIdx.x;
  const int L = 1 << lg;
  int Ns = 1;
  if (lg & 1) {
    constexpr int U = MAXE / (2 * NT);
    const int half = L >> 1;
    const int total = nl * half;
    Cx<R> a0[U], a1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = tid + u * NT;
      if (b < total) {
        const int l = b >> (lg - 1), j = b & (half - 1);
        a0[u] = buf[l * L + j];
        a1[u] = buf[l * L + j + half];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = tid + u * NT;
      if (b < total) {
        const int l = b >> (lg - 1), j = b & (half - 1);
        buf[l * L + 2 * j] = cadd(a0[u], a1[u]);
        buf[l * L + 2 * j + 1] = csub(a0[u], a1[u]);
      }
    }
    __syncthreads();
    Ns = 2;
  }
  constexpr int U = MAXE / (4 * NT);
  const int quarter = L >> 2;
  const int total = nl * quarter;
  for (; Ns < L; Ns <<= 2) {
    Cx<R> a[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = tid + u * NT;
      if (b < total) {
        const int l = b >> (lg - 2), j = b & (quarter - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) a[u][q] = buf[l * L + j + q * quarter];
      }
    }
    __syncthreads();
    const int tstep = L / (4 * Ns);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = tid + u * NT;
      if (b < total) {
        const int l = b >> (lg - 2), j = b & (quarter - 1);
        const int k = j & (Ns - 1);
        Cx<R> x0 = a[u][0], x1 = a[u][1], x2 = a[u][2], x3 = a[u][3];
        if (Ns > 1) {
          const Cx<R> w1 = twl[k * tstep];
          const Cx<R> w2 = cmul(w1, w1);
          const Cx<R> w3 = cmul(w2, w1);
          x1 = cmul(x1, w1);
          x2 = cmul(x2, w2);
          x3 = cmul(x3, w3);
        }
        const Cx<R> t0 = cadd(x0, x2), t1 = csub(x0, x2);
        const Cx<R> t2 = cadd(x1, x3), t3 = csub(x1, x3);
        const Cx<R> mt3 = {t3.y, -t3.x};  // -i * t3
        const int base = l * L + ((j - k) << 2) + k;
        buf[base] = cadd(t0, t2);
        buf[base + Ns] = cadd(t1, mt3);
        buf[base + 2 * Ns] = csub(t0, t2);
        buf[base + 3 * Ns] = csub(t1, mt3);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-wave FFT of lines of at most 256 points: a line of L = 2^lg points
// takes Q = L/4 lanes, one radix-4 Stockham butterfly per lane and stage (a
// radix-2 stage first when lg is odd), so a wave holds 256/L lines and needs
// no workgroup barrier.  A stage computes exactly what fft_lines computes
// for the same butterfly.
// ---------------------------------------------------------------------------
// Order the wave's own LDS accesses around an exchange between its lanes:
// LDS operations of one wave complete in issue order, so only the compiler
// has to be kept from moving them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane j enters with a[q] = x[j + q Q] and leaves with a[q] = X[j + q Q];
// the line occupies elements lo .. lo + L - 1 of wb, which holds the
// intermediate stages (written only when wr).  Reads of a stage precede its
// writes in issue order, so the line may be transformed in place.
template <typename R>
__device__ __forceinline__ void wave_fft_line(Cx<R> a[4], Cx<R> *wb, int lo, int j, int lg,
                                              const Cx<R> *twl, bool wr) {
  const int L = 1 << lg, Q = L >> 2;
  int Ns = 1;
  if (lg & 1) {
    // radix-2 stage: butterflies j and j + Q, of (x[b], x[b + L/2])
    wave_lds_sync();
    if (wr) {
      wb[lo + 2 * j] = cadd(a[0], a[2]);
      wb[lo + 2 * j + 1] = csub(a[0], a[2]);
      wb[lo + 2 * (j + Q)] = cadd(a[1], a[3]);
      wb[lo + 2 * (j + Q) + 1] = csub(a[1], a[3]);
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = wb[lo + j + q * Q];
    Ns = 2;
  }
  for (;; Ns <<= 2) {
    const int k = j & (Ns - 1);
    Cx<R> x0 = a[0], x1 = a[1], x2 = a[2], x3 = a[3];
    if (Ns > 1) {
      const Cx<R> w1 = twl[k * (L / (4 * Ns))];
      const Cx<R> w2 = cmul(w1, w1);
      const Cx<R> w3 = cmul(w2, w1);
      x1 = cmul(x1, w1);
      x2 = cmul(x2, w2);
      x3 = cmul(x3, w3);
    }
    const Cx<R> t0 = cadd(x0, x2), t1 = csub(x0, x2);
    const Cx<R> t2 = cadd(x1, x3), t3 = csub(x1, x3);
    const Cx<R> mt3 = {t3.y, -t3.x};   // -i t3
    a[0] = cadd(t0, t2);
    a[1] = cadd(t1, mt3);
    a[2] = csub(t0, t2);
    a[3] = csub(t1, mt3);
    // the last stage (Ns = Q) leaves output j + q Q in a[q]
    if (4 * Ns == L) break;
    const int base = lo + ((j - k) << 2) + k;
    wave_lds_sync();
    if (wr) {
#pragma unroll
      for (int q = 0; q < 4; ++q) wb[base + q * Ns] = a[q];
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = wb[lo + j + q * Q];
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// A tile of lines of one sine-transform pass.
// Element r of line l lives at global index base + l*lstride + r*stride.
// ---------------------------------------------------------------------------
struct LineTile {
  int ax;       // axis of the transform
  int n;        // line length (interior points along ax)
  int lg;       // log2 of the FFT length 2(n+1)
  int nl;       // valid lines in this tile
  int lp;       // lines per tile (power of two) of this pass
  int lgl;      // log2(lp)
  int base, stride, lstride;
  int row0;     // contiguous-axis passes: first row
  int outer;    // strided passes: index along the remaining axis (3-D)
  int c0;       // strided passes: first index along the contiguous axis
  uint32_t magic;  // ceil(2^32 / n), for e / n with e < 2^14
  // Column-blocked layout (block width B = 2^lgB): strided tiles address it
  // through base/stride/lstride directly (their lines are one block);
  // contiguous-axis tiles use qrow0 = row0 B and qblk = rows B, the offsets
  // of the tile's first row and of one block.
  int lgB, qrow0, qblk;
};

__device__ __forceinline__ int ilog2i(int v) { return 31 - __clz(v); }

__device__ __forceinline__ LineTile line_tile(const SysDesc &S, int ax, int lp, int tile) {
  LineTile t;
  t.ax = ax;
  t.n = S.n[ax];
  t.lg = S.lg[ax];
  t.lp = lp;
  t.lgl = ilog2i(t.lp);
  t.magic = (uint32_t)((0x100000000ull + (uint64_t)t.n - 1) / (uint64_t)t.n);
  t.lgB = S.lgB;
  t.qblk = S.rows << S.lgB;
  if (ax == S.d - 1) {
    t.row0 = tile * t.lp;
    t.nl = min(t.lp, S.rows - t.row0);
    t.base = t.row0 * t.n;
    t.stride = 1;
    t.lstride = t.n;
    t.outer = 0;
    t.c0 = 0;
    t.qrow0 = t.row0 << S.lgB;
  } else {
    // strided passes touch only column-blocked vectors: the tile's lp = B
    // lines c0 .. c0+B-1 are block c0 / B, element (l, r) of the tile at
    // ((c0 / B) rows + row(r)) B + l with row(r) the row index of position r
    const int nlast = S.n[S.d - 1];
    const int nblk = (nlast + t.lp - 1) / t.lp;
    const int outer = tile / nblk;
    const int blk = tile - outer * nblk;
    t.c0 = blk * t.lp;
    t.nl = min(t.lp, nlast - t.c0);
    t.outer = outer;
    // row(r) = rbase + r * rstep: 2-D axis 0: r; 3-D axis 1: outer n1 + r;
    // 3-D axis 0: r n1 + outer
    int rbase = 0, rstep = 1;
    if (S.d == 3) {
      if (ax == 1) rbase = outer * S.n[1];
      else {
        rbase = outer;
        rstep = S.n[1];
      }
    }
    t.base = (blk * S.rows + rbase) << S.lgB;
    t.stride = rstep << S.lgB;
    t.lstride = 1;
    t.row0 = 0;
    t.qrow0 = 0;
  }
  return t;
}

// Blocked order for contiguous-axis tiles reading or writing the
// column-blocked vectors: lanes run over W consecutive positions of a row,
// then the lp rows, then the next W positions, so a wave covers whole
// lp x B blocks (contiguous runs in memory) while its LDS accesses stay
// conflict-free (a row segment is 256 bytes of LDS).
// Returns the tile-local (line, position) and the blocked index q.
// With a block width of one (lgB = 0, planes of the two leading axes
// contiguous) the rows are the contiguous direction: lanes then run over the
// lp rows first.
template <int LGW>
__device__ __forceinline__ int tile_elems_blk(const LineTile &t) {
  if (t.lgB == 0) return t.n << t.lgl;
  return ((t.n + (1 << LGW) - 1) >> LGW) << (LGW + t.lgl);
}
template <int LGW>
__device__ __forceinline__ bool split_blk(const LineTile &t, int e, int &l, int &r, int &q) {
  if (t.lgB == 0) {
    l = e & (t.lp - 1);
    r = e >> t.lgl;
    q = r * t.qblk + t.qrow0 + l;
    return l < t.nl && r < t.n;
  }
  const int rl = e & ((1 << LGW) - 1);
  l = (e >> LGW) & (t.lp - 1);
  r = ((e >> (LGW + t.lgl)) << LGW) + rl;
  q = (r >> t.lgB) * t.qblk + t.qrow0 + (l << t.lgB) + (r & ((1 << t.lgB) - 1));
  return l < t.nl && r < t.n;
}
// row segment of 256 bytes: 16 FP64 or 32 FP32 complex entries
template <typename R> struct BlkW {
  static constexpr int lg = sizeof(R) == 8 ? 4 : 5;
};

// Split a flat element counter into (line, position).  Contiguous-axis
// tiles run positions fastest (coalesced rows); strided tiles run lines
// fastest (coalesced across adjacent lines).  Returns false if invalid.
__device__ __forceinline__ bool split_elem(const LineTile &t, int e, int &l, int &r) {
  if (t.stride == 1) {
    l = (int)__umulhi((uint32_t)e, t.magic);
    r = e - l * t.n;
    return l < t.nl;
  }
  r = e >> t.lgl;
  l = e & (t.lp - 1);
  return l < t.nl && r < t.n;
}

__device__ __forceinline__ int tile_elems(const LineTile &t) {
  return t.stride == 1 ? t.nl * t.n : t.lp * t.n;
}

// Fill the LDS lines with the odd extension [0, x_1..x_n, 0, -x_n..-x_1].
template <typename R, int U = 4, class Load>
__device__ __forceinline__ void lines_fill(Cx<R> *buf, const LineTile &t, Load &&load) {
  const int tid = threadIdx.x;
  const int L = 1 << t.lg, N = L >> 1;
  const int total = tile_elems(t);
  for (int e0 = 0; e0 < total; e0 += NT * U) {
    Cx<R> v[U];
    int pos[U], rr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT + tid;
      pos[u] = -1;
      int l, r;
      if (e < total && split_elem(t, e, l, r)) {
        v[u] = load(l, r, t.base + l * t.lstride + r * t.stride);
        pos[u] = l * L;
        rr[u] = r;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (pos[u] >= 0) {
        buf[pos[u] + rr[u] + 1] = v[u];
        buf[pos[u] + L - 1 - rr[u]] = Cx<R>{-v[u].x, -v[u].y};
      }
    }
  }
  for (int l = tid; l < t.nl; l += NT) {
    buf[l * L] = Cx<R>{0, 0};
    buf[l * L + N] = Cx<R>{0, 0};
  }
  __syncthreads();
}

// lines_fill for a contiguous-axis tile reading a column-blocked vector:
// load(l, r, q) with q the blocked index.
template <typename R, int U = 4, class Load>
__device__ __forceinline__ void lines_fill_blk(Cx<R> *buf, const LineTile &t, Load &&load) {
  const int tid = threadIdx.x;
  const int L = 1 << t.lg, N = L >> 1;
  constexpr int LGW = BlkW<R>::lg;
  const int total = tile_elems_blk<LGW>(t);
  for (int e0 = 0; e0 < total; e0 += NT * U) {
    Cx<R> v[U];
    int pos[U], rr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT + tid;
      pos[u] = -1;
      int l, r, q;
      if (e < total && split_blk<LGW>(t, e, l, r, q)) {
        v[u] = load(l, r, q);
        pos[u] = l * L;
        rr[u] = r;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (pos[u] >= 0) {
        buf[pos[u] + rr[u] + 1] = v[u];
        buf[pos[u] + L - 1 - rr[u]] = Cx<R>{-v[u].x, -v[u].y};
      }
    }
  }
  for (int l = tid; l < t.nl; l += NT) {
    buf[l * L] = Cx<R>{0, 0};
    buf[l * L + N] = Cx<R>{0, 0};
  }
  __syncthreads();
}

// Orthonormal DST-I output k = r + 1 of a transformed line:
// S_k = (i / sqrt(2N)) * Y_k.
template <typename R>
__device__ __forceinline__ Cx<R> dst_out(Cx<R> Y, R c) { return {-c * Y.y, c * Y.x}; }

// Scale the transformed lines mode by mode and re-extend them in place for
// the inverse transform (reads positions 1..N-1, writes N+1..2N-1 mirrors).
// Returns this thread's share of sum_k s_k |U_k|^2 over the tile, U the
// transform coefficients before scaling.
template <typename R, class Scale>
__device__ __forceinline__ double lines_scale_extend(Cx<R> *buf, const LineTile &t, Scale &&scale) {
  const int tid = threadIdx.x;
  const int L = 1 << t.lg, N = L >> 1;
  const R c = (R)1 / sqrt((R)L);
  const int total = tile_elems(t);
  double acc = 0.0;
  for (int e = tid; e < total; e += NT) {
    int l, r;
    if (split_elem(t, e, l, r)) {
      const int pos = l * L + r + 1;
      Cx<R> v = dst_out(buf[pos], c);
      const R s = scale(l, r);
      acc += (double)s * ((double)v.x * (double)v.x + (double)v.y * (double)v.y);
      v.x *= s;
      v.y *= s;
      buf[pos] = v;
      buf[l * L + L - 1 - r] = Cx<R>{-v.x, -v.y};
    }
  }
  for (int l = tid; l < t.nl; l += NT) {
    buf[l * L] = Cx<R>{0, 0};
    buf[l * L + N] = Cx<R>{0, 0};
  }
  __syncthreads();
  return acc;
}

template <typename R, class Store>
__device__ __forceinline__ void lines_store(const Cx<R> *buf, const LineTile &t, Store &&store) {
  const int tid = threadIdx.x;
  const int L = 1 << t.lg;
  const R c = (R)1 / sqrt((R)L);
  const int total = tile_elems(t);
  for (int e = tid; e < total; e += NT) {
    int l, r;
    if (split_elem(t, e, l, r)) {
      store(l, r, t.base + l * t.lstride + r * t.stride, dst_out(buf[l * L + r + 1], c));
    }
  }
  __syncthreads();
}

// lines_store for a contiguous-axis tile writing a column-blocked vector:
// store(l, r, q, value) with q the blocked index.
template <typename R, class Store>
__device__ __forceinline__ void lines_store_blk(const Cx<R> *buf, const LineTile &t, Store &&store) {
  const int tid = threadIdx.x;
  const int L = 1 << t.lg;
  const R c = (R)1 / sqrt((R)L);
  constexpr int LGW = BlkW<R>::lg;
  const int total = tile_elems_blk<LGW>(t);
  for (int e = tid; e < total; e += NT) {
    int l, r, q;
    if (split_blk<LGW>(t, e, l, r, q)) store(l, r, q, dst_out(buf[l * L + r + 1], c));
  }
  __syncthreads();
}

// Two-step variants: every global load of U elements (pre) is issued before
// any of them is consumed (make / post), so U elements' loads are in flight
// together.
template <typename R, int U, class Pre, class Make>
__device__ __forceinline__ void lines_fill2(Cx<R> *buf, const LineTile &t, Pre &&pre, Make &&make) {
  using PT = decltype(pre(0, 0, 0));
  const int tid = threadIdx.x;
  const int L = 1 << t.lg, N = L >> 1;
  const int total = tile_elems(t);
  // Two-deep software pipeline over rounds of NT*U elements: the loads of
  // the next round are in flight while this round is combined and written.
  struct Round {
    PT pv[U];
    int ll[U], rr[U], pp[U];
  };
  auto issue = [&](Round &q, int e0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT + tid;
      q.ll[u] = -1;
      int l, r;
      if (e < total && split_elem(t, e, l, r)) {
        q.ll[u] = l;
        q.rr[u] = r;
        q.pp[u] = t.base + l * t.lstride + r * t.stride;
        q.pv[u] = pre(l, r, q.pp[u]);
      }
    }
  };
  auto consume = [&](const Round &q) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (q.ll[u] >= 0) {
        const Cx<R> v = make(q.ll[u], q.rr[u], q.pp[u], q.pv[u]);
        buf[q.ll[u] * L + q.rr[u] + 1] = v;
        buf[q.ll[u] * L + L - 1 - q.rr[u]] = Cx<R>{-v.x, -v.y};
      }
    }
  };
  constexpr int step = NT * U;
  Round A, B;
  issue(A, 0);
  for (int e0 = 0; e0 < total; e0 += 2 * step) {
    if (e0 + step < total) issue(B, e0 + step);
    consume(A);
    if (e0 + step >= total) break;
    if (e0 + 2 * step < total) issue(A, e0 + 2 * step);
    consume(B);
  }
  for (int l = tid; l < t.nl; l += NT) {
    buf[l * L] = Cx<R>{0, 0};
    buf[l * L + N] = Cx<R>{0, 0};
  }
  __syncthreads();
}

template <typename R, int U, class Pre, class Post>
__device__ __forceinline__ void lines_store2(const Cx<R> *buf, const LineTile &t, Pre &&pre, Post &&post) {
  using PT = decltype(pre(0));
  const int tid = threadIdx.x;
  const int L = 1 << t.lg;
  const R c = (R)1 / sqrt((R)L);
  const int total = tile_elems(t);
  // same two-deep pipeline: the next round's operand loads are in flight
  // while this round is combined and stored
  struct Round {
    PT pv[U];
    int pp[U], bi[U];
  };
  auto issue = [&](Round &q, int e0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT + tid;
      q.pp[u] = -1;
      int l, r;
      if (e < total && split_elem(t, e, l, r)) {
        q.pp[u] = t.base + l * t.lstride + r * t.stride;
        q.bi[u] = l * L + r + 1;
        q.pv[u] = pre(q.pp[u]);
      }
    }
  };
  auto consume = [&](const Round &q) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (q.pp[u] >= 0) post(q.pp[u], dst_out(buf[q.bi[u]], c), q.pv[u]);
    }
  };
  constexpr int step = NT * U;
  Round A, B;
  issue(A, 0);
  for (int e0 = 0; e0 < total; e0 += 2 * step) {
    if (e0 + step < total) issue(B, e0 + step);
    consume(A);
    if (e0 + step >= total) break;
    if (e0 + 2 * step < total) issue(A, e0 + 2 * step);
    consume(B);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Stencil: (K u)_p = sum over the 2d faces e of p of c_e (u_p - u_nbr(e)) / h^2
// with u = 0 outside the grid.  The face coefficient is formed from the
// nodal samples a on the fly: the harmonic mean 2 a_p a_q / (a_p + a_q) of
// the two nodes of an interior face, the adjacent sample a_p on a boundary
// face.  The loads (u and a at p and its neighbours) are separated from the
// arithmetic so that pipelined fills can issue them early.
// ---------------------------------------------------------------------------
template <int D>
struct StencilIn {
  double2 c;          // u_p
  double2 b[D], a[D]; // neighbours below / above along each axis (0 outside)
  double ap;          // a_p
  double ab[D], aa[D];// a at those neighbours (a_p outside)
  unsigned inb, ina;  // bit ax: the neighbour below / above is inside
};

template <int D>
__device__ __forceinline__ StencilIn<D> stencil_load(const SysDesc &S,
                                                     const CSL_G double2 *__restrict__ u, int p,
                                                     const int (&idx)[3]) {
  StencilIn<D> in;
  const CSL_G double *__restrict__ A = gbl(S.a);
  in.c = ldg(u + p);
  in.ap = A[p];
  in.inb = 0u;
  in.ina = 0u;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    const int st = S.st[ax];
    const bool lo = idx[ax] > 0, hi = idx[ax] < S.n[ax] - 1;
    in.inb |= (lo ? 1u : 0u) << ax;
    in.ina |= (hi ? 1u : 0u) << ax;
    in.b[ax] = lo ? ldg(u + (p - st)) : make_double2(0.0, 0.0);
    in.a[ax] = hi ? ldg(u + (p + st)) : make_double2(0.0, 0.0);
    in.ab[ax] = lo ? A[p - st] : 0.0;
    in.aa[ax] = hi ? A[p + st] : 0.0;
  }
  return in;
}

// c_e / h^2 of the face between nodes with samples lo (lower index) and hi,
// or of a boundary face next to a node with sample ap
__device__ __forceinline__ double face_coef(bool inside, double lo, double hi, double ap, double h2) {
  const double c = inside ? 2.0 * lo * hi / (lo + hi) : ap;
  return c * h2;
}

template <int D>
__device__ __forceinline__ double2 stencil_apply(const SysDesc &S, const StencilIn<D> &in) {
  double rx = 0.0, ry = 0.0;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    const double h2 = S.h2[ax];
    const double fb = face_coef((in.inb >> ax) & 1u, in.ab[ax], in.ap, in.ap, h2);
    const double fa = face_coef((in.ina >> ax) & 1u, in.ap, in.aa[ax], in.ap, h2);
    rx += fb * (in.c.x - in.b[ax].x) + fa * (in.c.x - in.a[ax].x);
    ry += fb * (in.c.y - in.b[ax].y) + fa * (in.c.y - in.a[ax].y);
  }
  return make_double2(rx, ry);
}

template <int D>
__device__ __forceinline__ double2 stencil_K(const SysDesc &S, const CSL_G double2 *__restrict__ u,
                                             int p, const int (&idx)[3]) {
  return stencil_apply<D>(S, stencil_load<D>(S, u, p, idx));
}


// ---------------------------------------------------------------------------
// Dense sine-matrix transform on MFMA (lines of up to 1022 points).
// A chunk of lp complex lines is the real matrix X (np x 2 lp, np = n
// rounded up to 16; column 2l = Re of line l, 2l+1 = Im) stored in LDS as
// complex lines of np entries.  Y = W X with W the orthonormal DST-I matrix,
// which satisfies W[n-1-m][k] = (-1)^k W[m][k]: for the first h = ceil(n/2)
// rows, E = sum over even k and O = sum over odd k give Y[m] = E + O and
// Y[n-1-m] = E - O, half the products and half the matrix reads of the
// plain product.  The matrix is stored as two hp x hp blocks (hp = h rounded
// up to 16; global memory, zero padded): We[m][j] = W[m][2j] followed by
// Wo[m][j] = W[m][2j+1].  16x16x4 MFMA tiles: lane l feeds A[l%16][l/16]
// and B[l/16][l%16]; the accumulator row of register r is 4r + l/16 (FP64)
// or 4(l/16) + r (FP32), its column l%16.  X rows n..np-1 are never read and
// Y rows n..np-1 never written.
// ---------------------------------------------------------------------------
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
template <> struct Mfma<double> {
  typedef mfma_d4 acc;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lane) { return 4 * r + (lane >> 4); }
};
template <> struct Mfma<float> {
  typedef mfma_f4 acc;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lane) { return 4 * (lane >> 4) + r; }
};

__device__ __forceinline__ int gemm_np(int n) { return (n + 15) & ~15; }
__device__ __forceinline__ int gemm_hp(int n) { return (((n + 1) >> 1) + 15) & ~15; }

// Y = W X for a chunk of lp lines of n points, padded length np (X, Y in
// LDS).  The real and imaginary parts of a line are two columns of X; each
// wave owns 16 x 16 output blocks of the first h rows and streams the even
// and odd halves of K in steps of 4, taking W from the cache hierarchy and X
// from LDS.
template <typename R>
__device__ __forceinline__ void gemm_lines(const Cx<R> *X, Cx<R> *Y, int n, int np, int lp,
                                           const R *__restrict__ W) {
  constexpr int KU = 4;   // K steps in flight per half
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = (n + 1) >> 1, hp = gemm_hp(n);
  const int nrb = hp >> 4;
  const int ncb = (2 * lp + 15) >> 4;
  const int kq = hp >> 2;   // multiple of KU since hp is a multiple of 16
  const R *Xr = reinterpret_cast<const R *>(X);
  R *Yr = reinterpret_cast<R *>(Y);
  const int kl = lane >> 4;
  for (int blk = wave; blk < nrb * ncb; blk += NT / 64) {
    const int rb = blk / ncb, cb = blk - rb * ncb;
    const int m = rb * 16 + (lane & 15);
    const int col = cb * 16 + (lane & 15);
    const bool valid = col < 2 * lp;
    const int line = valid ? (col >> 1) : 0, part = col & 1;
    const CSL_G R *we = gbl(W) + m * hp + kl;
    const CSL_G R *wo = we + hp * hp;
    // even k = 2 (kl + 4 s), odd k = that + 1; element k of the line at 2k
    const R *xe = Xr + (line * np + 2 * kl) * 2 + part;
    typename Mfma<R>::acc ce = {0, 0, 0, 0}, co = {0, 0, 0, 0};
    for (int kk = 0; kk < kq; kk += KU) {
      R ae[KU], ao[KU], be[KU], bo[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = 2 * kl + 8 * (kk + u);
        ae[u] = we[(kk + u) * 4];
        ao[u] = wo[(kk + u) * 4];
        be[u] = (valid && k < n) ? xe[(kk + u) * 16] : (R)0;
        bo[u] = (valid && k + 1 < n) ? xe[(kk + u) * 16 + 2] : (R)0;
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        ce = Mfma<R>::step(ae[u], be[u], ce);
        co = Mfma<R>::step(ao[u], bo[u], co);
      }
    }
    if (valid) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mr = rb * 16 + Mfma<R>::row(r, lane);
        if (mr < h) {
          Yr[(line * np + mr) * 2 + part] = ce[r] + co[r];
          const int mm = n - 1 - mr;
          if (mm != mr) Yr[(line * np + mm) * 2 + part] = ce[r] - co[r];
        }
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// The same half-matrix product with FP16 matrix-core operations: operands
// split into high and low FP16 parts, x = xh + xl, W = Wh + Wl, and
// W x ~ Wh xh + Wh xl + Wl xh accumulated in FP32 (the dropped Wl xl is of
// order 2^-22 relative), which keeps the product at FP32 accuracy.  FP16
// has a narrow exponent range, so every column of X (the real or imaginary
// part of one line) is scaled by a power of two that puts its largest
// magnitude in [2^14, 2^15) before the split, and W is stored pre-scaled
// by 2^kGemm16Shift; both scales are exact and undone on output.  Stored
// matrix: four hp x hp FP16 blocks, Weh, Woh, Wel, Wol (even / odd columns
// of the first h rows, high / low parts).  16x16x16 f16 tiles: lane l feeds
// A[l%16][4(l/16) + j] and B[4(l/16) + j][l%16], j < 4; the accumulator row
// of register r is 4(l/16) + r, its column l%16.
// ---------------------------------------------------------------------------
typedef _Float16 mfma_h4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_h(float x, _Float16 &hi, _Float16 &lo) {
  hi = (_Float16)x;
  lo = (_Float16)(x - (float)hi);
}

// Exponent e per column of the chunk (2 lp columns: re and im of each line)
// such that max |x| 2^e lies in [2^14, 2^15); 0 for an all-zero column.
__device__ __forceinline__ void gemm16_col_scales(const Cx<float> *X, int n, int np, int lp,
                                                  int *colexp) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int l = wave; l < lp; l += NT / 64) {
    float mr = 0.f, mi = 0.f;
    for (int k = lane; k < n; k += 64) {
      const Cx<float> v = X[l * np + k];
      mr = fmaxf(mr, fabsf(v.x));
      mi = fmaxf(mi, fabsf(v.y));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      mr = fmaxf(mr, __shfl_xor(mr, off, 64));
      mi = fmaxf(mi, __shfl_xor(mi, off, 64));
    }
    if (lane == 0) {
      int er = 0, ei = 0;
      if (mr > 0.f) (void)frexpf(mr, &er);   // mr = m 2^er, m in [0.5, 1)
      if (mi > 0.f) (void)frexpf(mi, &ei);
      colexp[2 * l] = mr > 0.f ? 15 - er : 0;
      colexp[2 * l + 1] = mi > 0.f ? 15 - ei : 0;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void gemm_lines16(const Cx<float> *X, Cx<float> *Y, int n, int np,
                                             int lp, const _Float16 *__restrict__ W) {
  __shared__ int colexp[128];
  gemm16_col_scales(X, n, np, lp, colexp);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = (n + 1) >> 1, hp = gemm_hp(n);
  const int nrb = hp >> 4;
  const int ncb = (2 * lp + 15) >> 4;
  const int kb = hp >> 4;   // K blocks of 16
  const float *Xr = reinterpret_cast<const float *>(X);
  float *Yr = reinterpret_cast<float *>(Y);
  const int kl = lane >> 4;
  const size_t blk2 = (size_t)hp * hp;
  for (int blk = wave; blk < nrb * ncb; blk += NT / 64) {
    const int rb = blk / ncb, cb = blk - rb * ncb;
    const int m = rb * 16 + (lane & 15);
    const int col = cb * 16 + (lane & 15);
    const bool valid = col < 2 * lp;
    const int line = valid ? (col >> 1) : 0, part = col & 1;
    const int e = valid ? colexp[col] : 0;
    const float sc = ldexpf(1.0f, e);
    const CSL_G _Float16 *weh = gbl(W) + (size_t)m * hp + 4 * kl;
    const CSL_G _Float16 *woh = weh + blk2;
    const CSL_G _Float16 *wel = weh + 2 * blk2;
    const CSL_G _Float16 *wol = weh + 3 * blk2;
    // element k of the line sits at float index 2 k (re) or 2 k + 1 (im)
    const float *xl = Xr + (size_t)line * np * 2 + part;
    mfma_f4 ce = {0, 0, 0, 0}, co = {0, 0, 0, 0};
    for (int kk = 0; kk < kb; ++kk) {
      const mfma_h4 aeh = *(const CSL_G mfma_h4 *)(weh + kk * 16);
      const mfma_h4 aoh = *(const CSL_G mfma_h4 *)(woh + kk * 16);
      const mfma_h4 ael = *(const CSL_G mfma_h4 *)(wel + kk * 16);
      const mfma_h4 aol = *(const CSL_G mfma_h4 *)(wol + kk * 16);
      mfma_h4 beh, bel, boh, bol;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ke = 2 * (kk * 16 + 4 * kl + j);   // even k; the odd one is ke + 1
        const float xe = (valid && ke < n) ? xl[2 * ke] * sc : 0.f;
        const float xo = (valid && ke + 1 < n) ? xl[2 * ke + 2] * sc : 0.f;
        _Float16 hh, ll;
        split_h(xe, hh, ll);
        beh[j] = hh;
        bel[j] = ll;
        split_h(xo, hh, ll);
        boh[j] = hh;
        bol[j] = ll;
      }
      ce = __builtin_amdgcn_mfma_f32_16x16x16f16(ael, beh, ce, 0, 0, 0);
      ce = __builtin_amdgcn_mfma_f32_16x16x16f16(aeh, bel, ce, 0, 0, 0);
      ce = __builtin_amdgcn_mfma_f32_16x16x16f16(aeh, beh, ce, 0, 0, 0);
      co = __builtin_amdgcn_mfma_f32_16x16x16f16(aol, boh, co, 0, 0, 0);
      co = __builtin_amdgcn_mfma_f32_16x16x16f16(aoh, bol, co, 0, 0, 0);
      co = __builtin_amdgcn_mfma_f32_16x16x16f16(aoh, boh, co, 0, 0, 0);
    }
    if (valid) {
      const float us = ldexpf(1.0f, -(e + kGemm16Shift));
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mr = rb * 16 + 4 * kl + r;
        if (mr < h) {
          Yr[((size_t)line * np + mr) * 2 + part] = (ce[r] + co[r]) * us;
          const int mm = n - 1 - mr;
          if (mm != mr) Yr[((size_t)line * np + mm) * 2 + part] = (ce[r] - co[r]) * us;
        }
      }
    }
  }
  __syncthreads();
}

// Transform engines: the same tile code drives the LDS FFT (FftEng) or the
// MFMA sine-matrix product (GemmEng).
template <typename R, int LDSB> struct FftEng {
  static __device__ __forceinline__ const R *matrix(const SysDesc &, int) { return nullptr; }
  template <int U, class Load>
  static __device__ __forceinline__ void fill(Cx<R> *buf, const LineTile &t, Load &&load) {
    lines_fill<R, U>(buf, t, load);
  }
  template <int U, class Pre, class Make>
  static __device__ __forceinline__ void fill2(Cx<R> *buf, const LineTile &t, Pre &&pre,
                                               Make &&make) {
    lines_fill2<R, U>(buf, t, pre, make);
  }
  static __device__ __forceinline__ Cx<R> *transform(Cx<R> *buf, const LineTile &t,
                                                     const Cx<R> *twl, const R *) {
    fft_lines<R, LDSB>(buf, t.nl, t.lg, twl);
    return buf;
  }
  template <class Scale>
  static __device__ __forceinline__ double scale_transform(Cx<R> *buf, const LineTile &t,
                                                           const Cx<R> *twl, const R *,
                                                           Scale &&sc, Cx<R> **out) {
    const double acc = lines_scale_extend<R>(buf, t, sc);
    fft_lines<R, LDSB>(buf, t.nl, t.lg, twl);
    *out = buf;
    return acc;
  }
  template <class Store>
  static __device__ __forceinline__ void store(const Cx<R> *out, const LineTile &t, Store &&st) {
    lines_store<R>(out, t, st);
  }
  template <int U, class Pre, class Post>
  static __device__ __forceinline__ void store2(const Cx<R> *out, const LineTile &t, Pre &&pre,
                                                Post &&post) {
    lines_store2<R, U>(out, t, pre, post);
  }
  // contiguous-axis tiles on column-blocked vectors
  template <int U, class Load>
  static __device__ __forceinline__ void fill_blk(Cx<R> *buf, const LineTile &t, Load &&load) {
    lines_fill_blk<R, U>(buf, t, load);
  }
  template <class Store>
  static __device__ __forceinline__ void store_blk(const Cx<R> *out, const LineTile &t,
                                                   Store &&st) {
    lines_store_blk<R>(out, t, st);
  }
};


template <typename R, int LDSB> struct GemmEng {
  static __device__ __forceinline__ const R *matrix(const SysDesc &S, int ax) {
    if constexpr (sizeof(R) == 8) return reinterpret_cast<const R *>(S.Wm[ax]);
    else return reinterpret_cast<const R *>(S.Wmf[ax]);
  }
  template <int U, class Load>
  static __device__ __forceinline__ void fill(Cx<R> *buf, const LineTile &t, Load &&load) {
    const int np = gemm_np(t.n);
    const int total = tile_elems(t);
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < total; e0 += NT * U) {
      Cx<R> v[U];
      int pos[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * NT + tid;
        pos[u] = -1;
        int l, r;
        if (e < total && split_elem(t, e, l, r)) {
          v[u] = load(l, r, t.base + l * t.lstride + r * t.stride);
          pos[u] = l * np + r;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (pos[u] >= 0) buf[pos[u]] = v[u];
    }
    pad(buf, t, np);
  }
  template <int U, class Pre, class Make>
  static __device__ __forceinline__ void fill2(Cx<R> *buf, const LineTile &t, Pre &&pre,
                                               Make &&make) {
    using PT = decltype(pre(0, 0, 0));
    const int np = gemm_np(t.n);
    const int total = tile_elems(t);
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < total; e0 += NT * U) {
      PT pv[U];
      int ll[U], rr[U], pp[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * NT + tid;
        ll[u] = -1;
        int l, r;
        if (e < total && split_elem(t, e, l, r)) {
          ll[u] = l;
          rr[u] = r;
          pp[u] = t.base + l * t.lstride + r * t.stride;
          pv[u] = pre(l, r, pp[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ll[u] >= 0) buf[ll[u] * np + rr[u]] = make(ll[u], rr[u], pp[u], pv[u]);
    }
    pad(buf, t, np);
  }
  // zero the padding rows and the unused lines of the chunk
  static __device__ __forceinline__ void pad(Cx<R> *buf, const LineTile &t, int np) {
    const int padr = np - t.n;
    for (int e = threadIdx.x; e < t.lp * np; e += NT) {
      const int l = e / np, r = e - l * np;
      if (l >= t.nl || r >= t.n) buf[e] = Cx<R>{0, 0};
    }
    (void)padr;
    __syncthreads();
  }
  static __device__ __forceinline__ Cx<R> *transform(Cx<R> *buf, const LineTile &t,
                                                     const Cx<R> *, const R *W) {
    const int np = gemm_np(t.n);
    Cx<R> *Y = buf + t.lp * np;
    gemm_lines<R>(buf, Y, t.n, np, t.lp, W);
    return Y;
  }
  template <class Scale>
  static __device__ __forceinline__ double scale_transform(Cx<R> *buf, const LineTile &t,
                                                           const Cx<R> *, const R *W, Scale &&sc,
                                                           Cx<R> **out) {
    const int np = gemm_np(t.n);
    Cx<R> *Y = buf + t.lp * np;
    double acc = 0.0;
    const int total = tile_elems(t);
    for (int e = threadIdx.x; e < total; e += NT) {
      int l, r;
      if (split_elem(t, e, l, r)) {
        Cx<R> v = Y[l * np + r];
        const R s = sc(l, r);
        acc += (double)s * ((double)v.x * (double)v.x + (double)v.y * (double)v.y);
        v.x *= s;
        v.y *= s;
        Y[l * np + r] = v;
      }
    }
    __syncthreads();
    gemm_lines<R>(Y, buf, t.n, np, t.lp, W);
    *out = buf;
    return acc;
  }
  template <class Store>
  static __device__ __forceinline__ void store(const Cx<R> *out, const LineTile &t, Store &&st) {
    const int np = gemm_np(t.n);
    const int total = tile_elems(t);
    for (int e = threadIdx.x; e < total; e += NT) {
      int l, r;
      if (split_elem(t, e, l, r)) st(l, r, t.base + l * t.lstride + r * t.stride, out[l * np + r]);
    }
    __syncthreads();
  }
  template <int U, class Load>
  static __device__ __forceinline__ void fill_blk(Cx<R> *buf, const LineTile &t, Load &&load) {
    const int np = gemm_np(t.n);
    constexpr int LGW = BlkW<R>::lg;
    const int total = tile_elems_blk<LGW>(t);
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < total; e0 += NT * U) {
      Cx<R> v[U];
      int pos[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * NT + tid;
        pos[u] = -1;
        int l, r, q;
        if (e < total && split_blk<LGW>(t, e, l, r, q)) {
          v[u] = load(l, r, q);
          pos[u] = l * np + r;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (pos[u] >= 0) buf[pos[u]] = v[u];
    }
    pad(buf, t, np);
  }
  template <class Store>
  static __device__ __forceinline__ void store_blk(const Cx<R> *out, const LineTile &t,
                                                   Store &&st) {
    const int np = gemm_np(t.n);
    constexpr int LGW = BlkW<R>::lg;
    const int total = tile_elems_blk<LGW>(t);
    for (int e = threadIdx.x; e < total; e += NT) {
      int l, r, q;
      if (split_blk<LGW>(t, e, l, r, q)) st(l, r, q, out[l * np + r]);
    }
    __syncthreads();
  }
  template <int U, class Pre, class Post>
  static __device__ __forceinline__ void store2(const Cx<R> *out, const LineTile &t, Pre &&pre,
                                                Post &&post) {
    using PT = decltype(pre(0));
    const int np = gemm_np(t.n);
    const int total = tile_elems(t);
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < total; e0 += NT * U) {
      PT pv[U];
      Cx<R> vv[U];
      int pp[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * NT + tid;
        pp[u] = -1;
        int l, r;
        if (e < total && split_elem(t, e, l, r)) {
          pp[u] = t.base + l * t.lstride + r * t.stride;
          pv[u] = pre(pp[u]);
          vv[u] = out[l * np + r];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (pp[u] >= 0) post(pp[u], vv[u], pv[u]);
    }
    __syncthreads();
  }
};

// The matrix-core engine with FP16 split products (FP32 preconditioner data):
// the fills, stores and scaling of GemmEng, the product of gemm_lines16.
template <int LDSB> struct GemmEng16 : GemmEng<float, LDSB> {
  static __device__ __forceinline__ const float *matrix(const SysDesc &S, int ax) {
    return reinterpret_cast<const float *>(S.Wmh[ax]);
  }
  static __device__ __forceinline__ Cx<float> *transform(Cx<float> *buf, const LineTile &t,
                                                         const Cx<float> *, const float *W) {
    const int np = gemm_np(t.n);
    Cx<float> *Y = buf + t.lp * np;
    gemm_lines16(buf, Y, t.n, np, t.lp, reinterpret_cast<const _Float16 *>(W));
    return Y;
  }
  template <class Scale>
  static __device__ __forceinline__ double scale_transform(Cx<float> *buf, const LineTile &t,
                                                           const Cx<float> *, const float *W,
                                                           Scale &&sc, Cx<float> **out) {
    const int np = gemm_np(t.n);
    Cx<float> *Y = buf + t.lp * np;
    double acc = 0.0;
    const int total = tile_elems(t);
    for (int e = threadIdx.x; e < total; e += NT) {
      int l, r;
      if (split_elem(t, e, l, r)) {
        Cx<float> v = Y[l * np + r];
        const float s = sc(l, r);
        acc += (double)s * ((double)v.x * (double)v.x + (double)v.y * (double)v.y);
        v.x *= s;
        v.y *= s;
        Y[l * np + r] = v;
      }
    }
    __syncthreads();
    gemm_lines16(Y, buf, t.n, np, t.lp, reinterpret_cast<const _Float16 *>(W));
    *out = buf;
    return acc;
  }
};

// Multi-index of element r of contiguous-axis row `row`.
template <int D>
__device__ __forceinline__ void row_index(const SysDesc &S, int row, int r, int (&idx)[3]) {
  if (D == 2) {
    idx[0] = row;
    idx[1] = r;
    idx[2] = 0;
  } else {
    const int i0 = row / S.n[1];
    idx[0] = i0;
    idx[1] = row - i0 * S.n[1];
    idx[2] = r;
  }
}

// Workgroup sum in a fixed order (bitwise reproducible): butterfly
// reduction inside each wave, then the NT/64 wave sums in order.
__device__ __forceinline__ double wg_sum(double v, double *red) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

// Coherent reads of control scalars written by other workgroups.
__device__ __forceinline__ double ld_ctl(const double *p) {
  const unsigned long long b = __hip_atomic_load(
      reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)b);
}
__device__ __forceinline__ int ld_ctl(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace CSL_KNS
}  // namespace csl
