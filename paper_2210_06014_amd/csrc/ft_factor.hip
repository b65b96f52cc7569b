// Factor pass: shared g per fiber, in-place chains, chunk maps, combine.
#include "ft_device.h"

namespace ft {
namespace {

typedef float floatx2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Factor pass.  Each element x of a row, in order:
//     w = prod_{n != m} C(n)[i_n, :],  g = B(m) w,  e = x - a.g,
//     a <- a + (-lr lam) a + (lr e) g                       (Eq. (9), (10))
// The decay is applied as an increment so that its rounding does not build
// up over long rows.
//
// Per batch of 16 elements the lanes of a row first gather the C rows of all
// 16 elements (phase 1, latency overlapped), then run the 16 dependent steps.
// Steps past the end of an item use w = 0 and no decay, which leaves every
// state unchanged, so the wavefront needs no divergent control flow.

// Byte offset of row i of a C table, unsigned 32-bit: plan creation refuses
// I_n * R * 4 >= 2^31, so the product never wraps.
template <int R, class T>
__device__ __forceinline__ uint32_t row_bytes(int32_t i) {
  return (uint32_t)i * (uint32_t)(R * sizeof(T));
}

// value at byte offset `off` of a C table (uniform base + 32-bit offset: the
// scalar-base addressing form)
template <class T>
__device__ __forceinline__ float at_byte(const T* base, uint32_t off) {
  return to_f(*reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off));
}

// ixb[k]: byte offset of element (lane t)'s row in the k-th other C table
template <int N, int R, class T>
__device__ __forceinline__ void gather_w(const CPtrs<N, T>& cp, const int (&ixb)[N > 1 ? N - 1 : 1], int l, int t0,
                                         int len, float (&w)[16][R >= 16 ? R / 16 : 1]) {
  constexpr int RE = R >= 16 ? R / 16 : 1;
  static_for<0, 16>([&](auto S) {
    constexpr int s = decltype(S)::value;
    uint32_t ib[N - 1];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) ib[k] = (uint32_t)bcast16i<s>(ixb[k]);
    const bool sv = (t0 + s) < len;
#pragma unroll
    for (int q = 0; q < RE; ++q) {
      const uint32_t rb = (uint32_t)((R >= 16 ? l + 16 * q : (l % R)) * sizeof(T));
      float prod = at_byte(cp.p[0], ib[0] + rb);
#pragma unroll
      for (int k = 1; k < N - 1; ++k) prod *= at_byte(cp.p[k], ib[k] + rb);
      w[s][q] = sv ? prod : 0.f;
    }
  });
}

// g = B(m) w for this lane's elements j = l + 16 e; w_r comes from lane r % 16.
template <int J, int R>
__device__ __forceinline__ void shared_g(const float (&Bw)[J >= 16 ? J / 16 : 1][R], const float (&ws)[R >= 16 ? R / 16 : 1],
                                         float (&g)[J >= 16 ? J / 16 : 1]) {
  constexpr int E = J >= 16 ? J / 16 : 1;
  constexpr int RE = R >= 16 ? R / 16 : 1;
  constexpr int RK = R >= 16 ? 16 : R;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    g[e] = 0.f;
#pragma unroll
    for (int q = 0; q < RE; ++q) dot_bcast<RK>(g[e], ws[q], &Bw[e][16 * q]);
  }
}

// The shared intermediate of Section 3.2: g_f = B(m) w_f once per mode-m
// fiber f (w_f = prod_{n != m} C(n)[i_n, :] is the same for every element of
// the fiber).  Same lane layout and operation order as the per-element path,
// so the factor pass gives the same bits either way.  Each 16-lane group takes
// fiber_batches batches of 16 fibers and issues all their gathers first (one
// batch when the gathered values of two would not fit in registers).
template <int N, int R>
constexpr int fiber_batches() {
  return (N - 1) * (R >= 16 ? R / 16 : 1) > 8 ? 1 : 2;
}

template <int N, int J, int R, class T>
__global__ __launch_bounds__(256) void k_fiber_g(const int32_t* __restrict__ fib_idx, int64_t nfib, CPtrs<N, T> cp,
                                                 const T* __restrict__ Bm, float* __restrict__ gfib) {
  constexpr int E = J >= 16 ? J / 16 : 1;
  constexpr int RE = R >= 16 ? R / 16 : 1;
  constexpr int FB = fiber_batches<N, R>();
  const int l = threadIdx.x & 15;
  const int64_t f00 = ((int64_t)blockIdx.x * 16 + (threadIdx.x >> 4)) * 16 * FB;
  float Bw[E][R];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = l + 16 * e;
#pragma unroll
    for (int r = 0; r < R; ++r) Bw[e][r] = j < J ? to_f(Bm[j * R + r]) : 0.f;
  }
  int len[FB];
  int ixb[FB][N - 1];
#pragma unroll
  for (int b = 0; b < FB; ++b) {
    const int64_t f0 = f00 + 16 * b;
    len[b] = (int)max<int64_t>(0, min<int64_t>(16, nfib - f0));
    const int64_t f = min(f0 + l, nfib - 1);
#pragma unroll
    for (int k = 0; k < N - 1; ++k)
      ixb[b][k] = len[b] > 0 ? (int)row_bytes<R, T>(fib_idx[(int64_t)k * nfib + f]) : 0;
  }
  float w[FB][16][RE];
#pragma unroll
  for (int b = 0; b < FB; ++b) gather_w<N, R, T>(cp, ixb[b], l, 0, len[b], w[b]);
#pragma unroll
  for (int b = 0; b < FB; ++b) {
    const int64_t f0 = f00 + 16 * b;
    static_for<0, 16>([&](auto S) {
      constexpr int s = decltype(S)::value;
      float g[E];
      shared_g<J, R>(Bw, w[b][s], g);
      if (s < len[b]) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int j = l + 16 * e;
          if (j < J) gfib[(f0 + s) * J + j] = g[e];
        }
      }
    });
  }
}

// Heads write the row's head vector, or A(m) itself when hvec is null (the
// relaxed passes).  With RLX the items are the chunks of long rows under
// FT_RELAXED: each runs from the row as its head left it, a_H (in A(m); the
// merge that follows is the only other writer) and stores its increment
// beyond the decay of a_H, weighted by the decay of the row's later elements,
//     rho^T (a - rho^len a_H),   T = elements of the row after the chunk,
// and the sum of ||g||^2 over its steps, J + 1 floats per chunk slot.
template <int N, int J, int R, class T, bool FIB, bool NC = false, bool RLX = false>
__device__ __forceinline__ void apply_item(int64_t gid, const FItem* __restrict__ items, int64_t n_items,
                                           const int32_t* __restrict__ idx, int64_t nnz, const float* __restrict__ val,
                                           const CPtrs<N, T>& cp, const T* __restrict__ Bm, float* __restrict__ Am,
                                           float* __restrict__ hvec, float lr, float c1,
                                           const int32_t* __restrict__ fid, const float* __restrict__ gfib,
                                           const NoC<N>& nc, float* __restrict__ incr,
                                           const int64_t* __restrict__ row_ptr, double rho) {
  constexpr int E = J >= 16 ? J / 16 : 1;
  constexpr int RE = R >= 16 ? R / 16 : 1;
  const int l = threadIdx.x & 15;
  float Bw[E][R];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = l + 16 * e;
#pragma unroll
    for (int r = 0; r < R; ++r) Bw[e][r] = (!FIB && j < J) ? to_f(Bm[j * R + r]) : 0.f;
  }
  static_assert(!NC || (J == 16 && R == 16 && !FIB), "the no-C-cache variant is built for J = R = 16");
  float Bc[N > 1 ? N - 1 : 1][16];
  if constexpr (NC) load_nc_cols<N>(nc, l, Bc);
  FItem it{0, 0, 0, 0, 0};
  if (gid < n_items) it = items[gid];
  // The row is carried in FP64 registers and rounded to FP32 once when
  // stored: the decay step lr*lam*a is about a hundred ulps of a, nearly the
  // same every step, so FP32 rounding of the running state would accumulate
  // coherently (up to k/2 ulps after k steps) instead of averaging out.
  double a[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = l + 16 * e;
    a[e] = (it.len > 0 && j < J) ? (double)Am[(int64_t)it.row * J + j] : 0.0;
  }
  int maxlen = it.len;
  maxlen = max(maxlen, __shfl_xor(maxlen, 16));
  maxlen = max(maxlen, __shfl_xor(maxlen, 32));
  // Software pipeline over batches of 16 elements: while the 16 dependent
  // steps of batch b run, the gathers of batch b + 1 and the index loads of
  // batch b + 2 are in flight, so a long serial item waits on arithmetic, not
  // on memory.  Past the end, positions clamp to the item's last element (a
  // valid address) and steps are neutralised (w = 0, no decay).
  constexpr int WD = FIB ? E : RE;
  constexpr int NI = N > 1 ? N - 1 : 1;
  auto stage_a = [&](int t0, float& xv, int (&ix)[NI]) {
    const int64_t p = it.start + min(t0 + l, max(it.len - 1, 0));
    xv = it.len > 0 ? val[p] : 0.f;
    if constexpr (FIB) {
      ix[0] = it.len > 0 ? fid[p] : 0;
    } else {
#pragma unroll
      for (int k = 0; k < N - 1; ++k)
        ix[k] = it.len > 0 ? (NC ? idx[(int64_t)k * nnz + p] : (int)row_bytes<R, T>(idx[(int64_t)k * nnz + p])) : 0;
    }
  };
  auto stage_b = [&](int t0, const int (&ix)[NI], float (&w)[16][WD]) {
    if constexpr (FIB) {
      static_for<0, 16>([&](auto S) {
        constexpr int s = decltype(S)::value;
        const int64_t fb = (int64_t)bcast16i<s>(ix[0]) * J;
        const bool sv = (t0 + s) < it.len;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          // unconditional load (a valid fiber, the column clamped) so that all
          // 16 loads are in flight together; masked afterwards
          const int j = l + 16 * e;
          const float gv = gfib[fb + min(j, J - 1)];
          w[s][e] = (sv && j < J) ? gv : 0.f;
        }
      });
    } else if constexpr (NC) {
      gather_w_nc<N>(nc, Bc, ix, l, t0, it.len, w);
    } else {
      gather_w<N, R, T>(cp, ix, l, t0, it.len, w);
    }
  };
  // (high orders keep one batch in registers: two would spill)
  constexpr bool PIPE = (N - 1) * WD <= 4;
  float gg = 0.f;  // sum of ||g||^2 over the steps (RLX)
  float xv0, xv1 = 0.f;
  int ix1[NI];
  float w0[16][WD];
  if constexpr (PIPE) {
    int ix0[NI];
    stage_a(0, xv0, ix0);
    stage_b(0, ix0, w0);
    stage_a(16, xv1, ix1);
  }
  for (int t0 = 0; t0 < maxlen; t0 += 16) {
    float wn[16][WD];
    float xv2 = 0.f;
    int ix2[NI];
    if constexpr (PIPE) {
      stage_b(t0 + 16, ix1, wn);
      stage_a(t0 + 32, xv2, ix2);
    } else {
      int ixc[NI];
      stage_a(t0, xv0, ixc);
      stage_b(t0, ixc, w0);
    }
    static_for<0, 16>([&](auto S) {
      constexpr int s = decltype(S)::value;
      float g[E];
      if constexpr (FIB) {
#pragma unroll
        for (int e = 0; e < E; ++e) g[e] = w0[s][e];
      } else {
        shared_g<J, R>(Bw, w0[s], g);
      }
      float pr = 0.f;
#pragma unroll
      for (int e = 0; e < E; ++e) pr = fmaf((float)a[e], g[e], pr);
      pr = group_sum<16>(pr);
      const float es = bcast16<s>(xv0) - pr;
      const double dec = (t0 + s) < it.len ? (double)c1 : 0.0;
      const double le = (double)(lr * es);
      if constexpr (RLX) {
#pragma unroll
        for (int e = 0; e < E; ++e) gg = fmaf(g[e], g[e], gg);  // g = 0 past the end
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        a[e] = fma(dec, a[e], a[e]);
        a[e] = fma(le, (double)g[e], a[e]);
      }
    });
    if constexpr (PIPE) {
#pragma unroll
      for (int s = 0; s < 16; ++s)
#pragma unroll
        for (int e = 0; e < WD; ++e) w0[s][e] = wn[s][e];
      xv0 = xv1;
      xv1 = xv2;
#pragma unroll
      for (int k = 0; k < NI; ++k) ix1[k] = ix2[k];
    }
  }
  if constexpr (RLX) {
    gg = group_sum<16>(gg);
    if (it.len > 0) {
      const double own = pow(rho, (double)it.len);
      const double after = pow(rho, (double)(row_ptr[it.row + 1] - (it.start + it.len)));
      float* dst = incr + (int64_t)it.slot * (J + 1);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int j = l + 16 * e;
        if (j < J) dst[j] = (float)(after * (a[e] - own * (double)Am[(int64_t)it.row * J + j]));
      }
      if (l == 0) dst[J] = gg;
    }
    return;
  }
  if (it.len > 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = l + 16 * e;
      if (j < J) {
        if (it.kind == ITEM_LIGHT || hvec == nullptr)
          Am[(int64_t)it.row * J + j] = (float)a[e];
        else
          hvec[(int64_t)it.slot * J + j] = (float)a[e];
      }
    }
  }
}

// One item per 16-lane group: the four groups of a wavefront take four
// consecutive items (similar lengths, the lists are sorted).
template <int N, int J, int R, class T, bool FIB, bool NC = false, bool RLX = false>
__global__ __launch_bounds__(256) void k_factor_apply(const FItem* __restrict__ items, int64_t n_items,
                                                      const int32_t* __restrict__ idx, int64_t nnz,
                                                      const float* __restrict__ val, CPtrs<N, T> cp,
                                                      const T* __restrict__ Bm, float* __restrict__ Am,
                                                      float* __restrict__ hvec, float lr, float c1,
                                                      const int32_t* __restrict__ fid, const float* __restrict__ gfib,
                                                      NoC<N> nc, float* __restrict__ incr,
                                                      const int64_t* __restrict__ row_ptr, double rho) {
  apply_item<N, J, R, T, FIB, NC, RLX>((int64_t)blockIdx.x * 16 + (threadIdx.x >> 4), items, n_items, idx, nnz, val,
                                       cp, Bm, Am, hvec, lr, c1, fid, gfib, nc, incr, row_ptr, rho);
}

// Chunk maps.  With rho = 1 - lr lam and gp = lr / rho, one step is
//     a <- rho (I - gp g g^T) a + lr x g.
// A chunk of T steps is the affine map a -> rho^T (I + Nm) a + v with
//     Nm <- Nm - gp g (g + Nm^T g)^T     (Nm = prod (I - gp g g^T) - I)
//     v  <- v + (-lr lam) v + lr (x - v.g) g
// (v is the state reached from a = 0).  Lane j keeps column j of Nm.
template <int N, int J, int R, class T, bool FIB, bool NC = false>
__device__ __forceinline__ void compose_item(int64_t gid, const FItem* __restrict__ items, int64_t n_items,
                                             const int32_t* __restrict__ idx, int64_t nnz,
                                             const float* __restrict__ val, const CPtrs<N, T>& cp,
                                             const T* __restrict__ Bm, float* __restrict__ maps,
                                             double* __restrict__ map_scale, float lr, float c1, float gp, double rho,
                                             const int32_t* __restrict__ fid, const float* __restrict__ gfib,
                                             const NoC<N>& nc) {
  constexpr int E = J >= 16 ? J / 16 : 1;
  constexpr int RE = R >= 16 ? R / 16 : 1;
  constexpr int MS = J * J + J;
  const int l = threadIdx.x & 15;
  float Bw[E][R];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = l + 16 * e;
#pragma unroll
    for (int r = 0; r < R; ++r) Bw[e][r] = (!FIB && j < J) ? to_f(Bm[j * R + r]) : 0.f;
  }
  static_assert(!NC || (J == 16 && R == 16 && !FIB), "the no-C-cache variant is built for J = R = 16");
  float Bc[N > 1 ? N - 1 : 1][16];
  if constexpr (NC) load_nc_cols<N>(nc, l, Bc);
  FItem it{0, 0, 0, 0, 0};
  if (gid < n_items) it = items[gid];
  float Nc[E][J];
  float v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = 0.f;
#pragma unroll
    for (int i = 0; i < J; ++i) Nc[e][i] = 0.f;
  }
  int maxlen = it.len;
  maxlen = max(maxlen, __shfl_xor(maxlen, 16));
  maxlen = max(maxlen, __shfl_xor(maxlen, 32));
  for (int t0 = 0; t0 < maxlen; t0 += 16) {
    // past the end: clamp to the item's last element (valid address); those
    // steps are neutralised below (w = 0, no decay)
    const int64_t p = it.start + min(t0 + l, max(it.len - 1, 0));
    const float xv = it.len > 0 ? val[p] : 0.f;
    // phase 1: w of the 16 elements (or, with fibers, their precomputed g)
    float w[16][FIB ? E : RE];
    if constexpr (FIB) {
      const int fv = it.len > 0 ? fid[p] : 0;
      static_for<0, 16>([&](auto S) {
        constexpr int s = decltype(S)::value;
        const int64_t fb = (int64_t)bcast16i<s>(fv) * J;
        const bool sv = (t0 + s) < it.len;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          // unconditional load (fv is a valid fiber, the column clamped) so
          // that all 16 loads are in flight together; masked afterwards
          const int j = l + 16 * e;
          const float gv = gfib[fb + min(j, J - 1)];
          w[s][e] = (sv && j < J) ? gv : 0.f;
        }
      });
    } else {
      int ix[N - 1];
#pragma unroll
      for (int k = 0; k < N - 1; ++k)
        ix[k] = it.len > 0 ? (NC ? idx[(int64_t)k * nnz + p] : (int)row_bytes<R, T>(idx[(int64_t)k * nnz + p])) : 0;
      if constexpr (NC)
        gather_w_nc<N>(nc, Bc, ix, l, t0, it.len, w);
      else
        gather_w<N, R, T>(cp, ix, l, t0, it.len, w);
    }
    static_for<0, 16>([&](auto S) {
      constexpr int s = decltype(S)::value;
      float g[E];
      if constexpr (FIB) {
#pragma unroll
        for (int e = 0; e < E; ++e) g[e] = w[s][e];
      } else {
        shared_g<J, R>(Bw, w[s], g);
      }
      constexpr int JK = J >= 16 ? 16 : J;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        // h = g_j + sum_i Nm[i][j] g_i ;  Nm[:, j] -= gp * h * g
        float h = g[e];
#pragma unroll
        for (int q = 0; q < E; ++q) dot_bcast<JK>(h, g[q], &Nc[e][16 * q]);
        const float t = -gp * h;
#pragma unroll
        for (int q = 0; q < E; ++q) axpy_bcast<JK>(&Nc[e][16 * q], g[q], t);
      }
      float pr = 0.f;
#pragma unroll
      for (int e = 0; e < E; ++e) pr = fmaf(v[e], g[e], pr);
      pr = group_sum<16>(pr);
      const float es = bcast16<s>(xv) - pr;
      const float dec = (t0 + s) < it.len ? c1 : 0.f;
      const float le = lr * es;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        v[e] = fmaf(dec, v[e], v[e]);
        v[e] = fmaf(le, g[e], v[e]);
      }
    });
  }
  if (it.len > 0) {
    float* dst = maps + (int64_t)it.slot * MS;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = l + 16 * e;
      if (j < J) {
#pragma unroll
        for (int i = 0; i < J; ++i) dst[j * J + i] = Nc[e][i];  // column-major
        dst[J * J + j] = v[e];
      }
    }
    if (l == 0) map_scale[it.slot] = pow(rho, (double)it.len);
  }
}

template <int N, int J, int R, class T, bool FIB, bool NC = false>
__global__ __launch_bounds__(256) void k_factor_compose(const FItem* __restrict__ items, int64_t n_items,
                                                        const int32_t* __restrict__ idx, int64_t nnz,
                                                        const float* __restrict__ val, CPtrs<N, T> cp,
                                                        const T* __restrict__ Bm, float* __restrict__ maps,
                                                        double* __restrict__ map_scale, float lr, float c1, float gp,
                                                        double rho, const int32_t* __restrict__ fid,
                                                        const float* __restrict__ gfib, NoC<N> nc) {
  compose_item<N, J, R, T, FIB, NC>((int64_t)blockIdx.x * 16 + (threadIdx.x >> 4), items, n_items, idx, nnz, val, cp,
                                    Bm, maps, map_scale, lr, c1, gp, rho, fid, gfib, nc);
}

// The in-place items and the chunk maps of one exact factor pass in one
// launch.  They are independent (a map starts from the identity, not from
// its row's head), so the first apply_blocks workgroups take the in-place
// items, heads of long rows first, and the rest the chunk maps: the long
// serial heads start at once and run while the maps keep the SIMDs busy,
// instead of running on an otherwise idle GPU after them.
template <int N, int J, int R, class T, bool FIB, bool NC = false>
__global__ __launch_bounds__(256) void k_factor_fused(int64_t apply_blocks, const FItem* __restrict__ apply_items,
                                                      int64_t n_apply, const FItem* __restrict__ compose_items,
                                                      int64_t n_compose, const int32_t* __restrict__ idx, int64_t nnz,
                                                      const float* __restrict__ val, CPtrs<N, T> cp,
                                                      const T* __restrict__ Bm, float* __restrict__ Am,
                                                      float* __restrict__ hvec, float* __restrict__ maps,
                                                      double* __restrict__ map_scale, float lr, float c1, float gp,
                                                      double rho, const int32_t* __restrict__ fid,
                                                      const float* __restrict__ gfib, NoC<N> nc) {
  const int64_t grp = threadIdx.x >> 4;
  if ((int64_t)blockIdx.x < apply_blocks)
    apply_item<N, J, R, T, FIB, NC, false>((int64_t)blockIdx.x * 16 + grp, apply_items, n_apply, idx, nnz, val, cp,
                                           Bm, Am, hvec, lr, c1, fid, gfib, nc, nullptr, nullptr, rho);
  else
    compose_item<N, J, R, T, FIB, NC>(((int64_t)blockIdx.x - apply_blocks) * 16 + grp, compose_items, n_compose, idx,
                                      nnz, val, cp, Bm, maps, map_scale, lr, c1, gp, rho, fid, gfib, nc);
}

// Fold `count` consecutive maps (earliest first) into one, as a binary tree in
// LDS (fixed bracketing: pairs (0,1), (2,3), ... then (0,2), ... so that a
// later map is always applied after an earlier one):
//   (s2, N2, v2) o (s1, N1, v1) = (s1 s2, N1 + N2 + N2 N1, s2 (v1 + N2 v1) + v2),
// with s = rho^length kept in FP64.  Only rows with more maps than the last
// fold takes in sequence (below) pass through here.
template <int J>
constexpr int combine_fanin() {
  return J <= 16 ? 16 : 8;  // maps held in LDS by one workgroup
}

template <int J>
__global__ __launch_bounds__(256) void k_combine(const CItem* __restrict__ items, float* __restrict__ maps,
                                                 double* __restrict__ map_scale) {
  constexpr int MS = J * J + J;
  constexpr int F = combine_fanin<J>();
  // a thread forms a T x T tile of a product: 4 x 4 at J = 32, 2 x 2 at
  // J = 16 (fan-in 16: 512 tiles for the 256 threads), one entry at J = 8
  constexpr int T = J >= 32 ? 4 : J >= 16 ? 2 : 1;
  constexpr int T4 = J / T;                            // output tiles per side of a product
  constexpr int TMAX = (F / 2 * T4 * T4 + 255) / 256;  // output tiles per thread at the widest level
  constexpr int VMAX = (F / 2 * J + 255) / 256;        // vector entries per thread at the widest level
  static_assert(J % 4 == 0 && MS % 4 == 0, "16-byte LDS reads of map columns");
  __shared__ __align__(16) float buf[F * MS];
  __shared__ double sc[F];
  const CItem it = items[blockIdx.x];
  const int t = threadIdx.x;
  const int count = it.count;
  {
    const float* src = maps + it.in_off * MS;
    for (int k = t; k < count * MS; k += 256) buf[k] = src[k];
    if (t < count) sc[t] = map_scale[it.in_off + t];
  }
  __syncthreads();
  for (int stride = 1; stride < count; stride *= 2) {
    const int pairs = (count - stride + 2 * stride - 1) / (2 * stride);  // a = 2 k stride, b = a + stride < count
    // (N_b N_a)(i, j) = sum_q N_b(i, q) N_a(q, j), q in order, for a T x T
    // tile of (i, j) per thread.  Columns are contiguous (entry (i, j) at
    // j J + i), so each step of four q reads T columns of N_a (16 bytes
    // each) and four column pieces of N_b (4 T bytes each) for 4 T^2 FMAs.
    float res[TMAX][T][T];
#pragma unroll
    for (int u = 0; u < TMAX; ++u) {
      const int e = t + 256 * u;
      if (e < pairs * T4 * T4) {
        const int pr = e / (T4 * T4), rem = e % (T4 * T4);
        const int i0 = T * (rem % T4), j0 = T * (rem / T4);
        const float* Na = buf + (2 * pr * stride) * MS;
        const float* Nb = Na + stride * MS;
        if constexpr (T == 1) {
          float acc = 0.f;
#pragma unroll
          for (int q = 0; q < J; ++q) acc = fmaf(Nb[q * J + i0], Na[j0 * J + q], acc);
          const int ij = j0 * J + i0;
          res[u][0][0] = (Na[ij] + Nb[ij]) + acc;
        } else {
          using Vec = typename std::conditional<T == 4, floatx4, floatx2>::type;
          float acc[T][T];  // acc[c][r]: entry (i0 + r, j0 + c)
#pragma unroll
          for (int c = 0; c < T; ++c)
#pragma unroll
            for (int r = 0; r < T; ++r) acc[c][r] = 0.f;
#pragma unroll
          for (int q0 = 0; q0 < J; q0 += 4) {
            floatx4 na[T];
            Vec nb[4];
#pragma unroll
            for (int c = 0; c < T; ++c) na[c] = *reinterpret_cast<const floatx4*>(Na + (j0 + c) * J + q0);
#pragma unroll
            for (int k = 0; k < 4; ++k) nb[k] = *reinterpret_cast<const Vec*>(Nb + (q0 + k) * J + i0);
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
              for (int c = 0; c < T; ++c)
#pragma unroll
                for (int r = 0; r < T; ++r) acc[c][r] = fmaf(nb[k][r], na[c][k], acc[c][r]);
          }
#pragma unroll
          for (int c = 0; c < T; ++c)
#pragma unroll
            for (int r = 0; r < T; ++r) {
              const int ij = (j0 + c) * J + i0 + r;
              res[u][c][r] = (Na[ij] + Nb[ij]) + acc[c][r];
            }
        }
      }
    }
    float vres[VMAX];
    double sres[VMAX];
#pragma unroll
    for (int u = 0; u < VMAX; ++u) {
      const int e = t + 256 * u;
      if (e < pairs * J) {
        const int pr = e / J, i = e % J;
        const float* Na = buf + (2 * pr * stride) * MS;
        const float* Nb = Na + stride * MS;
        float acc = 0.f;
#pragma unroll
        for (int q = 0; q < J; ++q) acc = fmaf(Nb[q * J + i], Na[J * J + q], acc);
        const double sb = sc[2 * pr * stride + stride];
        vres[u] = (float)(sb * ((double)Na[J * J + i] + (double)acc)) + Nb[J * J + i];
        sres[u] = sc[2 * pr * stride] * sb;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < TMAX; ++u) {
      const int e = t + 256 * u;
      if (e < pairs * T4 * T4) {
        const int pr = e / (T4 * T4), rem = e % (T4 * T4);
        const int i0 = T * (rem % T4), j0 = T * (rem / T4);
#pragma unroll
        for (int c = 0; c < T; ++c)
#pragma unroll
          for (int r = 0; r < T; ++r) buf[(2 * pr * stride) * MS + (j0 + c) * J + i0 + r] = res[u][c][r];
      }
    }
#pragma unroll
    for (int u = 0; u < VMAX; ++u) {
      const int e = t + 256 * u;
      if (e < pairs * J) {
        const int pr = e / J, i = e % J;
        buf[(2 * pr * stride) * MS + J * J + i] = vres[u];
        if (i == 0) sc[2 * pr * stride] = sres[u];
      }
    }
    __syncthreads();
  }
  float* dst = maps + it.out_off * MS;
  for (int k = t; k < MS; k += 256) dst[k] = buf[k];
  if (t == 0) map_scale[it.out_off] = sc[0];
}

// Last fold of a heavy row: its remaining maps, earliest first, applied to
// the head vector (the row's state after its first chunk),
//     a <- s (a + N a) + v,
// J^2 work per map where composing two maps costs J^3.  One 16-lane group
// per row; lane i holds a_i in FP64 and row i of the maps in flight (D of
// them, loaded ahead of the dependent chain).  Rows of a wavefront have
// similar map counts (the list is sorted by count); steps past a row's count
// leave it unchanged.
template <int J>
__global__ __launch_bounds__(256) void k_combine_final(const CItem* __restrict__ items, int64_t n_items,
                                                       const float* __restrict__ maps,
                                                       const double* __restrict__ map_scale,
                                                       const float* __restrict__ hvec, float* __restrict__ Am) {
  constexpr int E = J >= 16 ? J / 16 : 1;
  constexpr int K = J >= 16 ? 16 : J;
  constexpr int MS = J * J + J;
  constexpr int D = J >= 32 ? 2 : 4;
  const int l = threadIdx.x & 15;
  const int64_t gid = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  CItem it{0, 0, 0, 0, 0, 0};
  if (gid < n_items) it = items[gid];
  double a[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = l + 16 * e;
    a[e] = (it.count > 0 && j < J) ? (double)hvec[(int64_t)it.heavy * J + j] : 0.0;
  }
  int maxc = it.count;
  maxc = max(maxc, __shfl_xor(maxc, 16));
  maxc = max(maxc, __shfl_xor(maxc, 32));
  // row i = l + 16 e of map k (entry (i, q) at q J + i); lanes past J (J = 8)
  // read row J - 1 and discard it.  Past the row's count: its last map.
  auto load = [&](int k, float (&Nr)[E][J], float (&v)[E], double& sc) {
    const int64_t slot = it.in_off + min(k, max(it.count - 1, 0));
    const float* mp = maps + slot * MS;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = min(l + 16 * e, J - 1);
#pragma unroll
      for (int q = 0; q < J; ++q) Nr[e][q] = mp[q * J + i];
      v[e] = mp[J * J + i];
    }
    sc = map_scale[slot];
  };
  float Nq[D][E][J], vq[D][E];
  double sq[D];
  static_for<0, D>([&](auto S) { load(decltype(S)::value, Nq[decltype(S)::value], vq[decltype(S)::value],
                                      sq[decltype(S)::value]); });
  for (int k0 = 0; k0 < maxc; k0 += D) {
    static_for<0, D>([&](auto S) {
      constexpr int d = decltype(S)::value;
      const int k = k0 + d;
      if (k < maxc) {
        float af[E];
#pragma unroll
        for (int e = 0; e < E; ++e) af[e] = (float)a[e];
        float acc[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          acc[e] = 0.f;
#pragma unroll
          for (int e2 = 0; e2 < E; ++e2) dot_bcast<K>(acc[e], af[e2], &Nq[d][e][16 * e2]);
        }
        if (k < it.count) {
#pragma unroll
          for (int e = 0; e < E; ++e) a[e] = sq[d] * (a[e] + (double)acc[e]) + (double)vq[d][e];
        }
        load(k + D, Nq[d], vq[d], sq[d]);
      }
    });
  }
  if (it.count > 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = l + 16 * e;
      if (j < J) Am[(int64_t)it.row * J + j] = (float)a[e];
    }
  }
}

// FT_RELAXED merge of a long row's chunk increments, in two fixed levels so
// that rows of many thousand chunks spread over many workgroups and the sums
// do not depend on timing.  Both levels sum `count` consecutive records of
// J + 1 values (the increment, then sum ||g||^2) in FP64: thread (sub, j)
// adds records sub, sub + S, sub + 2 S, ... (S = 256 / J; a wavefront reads
// 64 / J consecutive records, one contiguous run), then the S partial sums
// are added in a fixed tree order in LDS.
template <int J, class In>
__device__ __forceinline__ void sum_records(const In* __restrict__ base, int count, double (&ssum)[256 / J][J + 1]) {
  constexpr int S = 256 / J;
  const int t = threadIdx.x, j = t % J, sub = t / J;
  double s = 0.0, G = 0.0;
#pragma unroll 4
  for (int k = sub; k < count; k += S) {
    s += (double)base[(int64_t)k * (J + 1) + j];
    if (j == 0) G += (double)base[(int64_t)k * (J + 1) + J];
  }
  ssum[sub][j] = s;
  if (j == 0) ssum[sub][J] = G;
  __syncthreads();
  for (int stride = S / 2; stride >= 1; stride /= 2) {
    if (sub < stride) {
      ssum[sub][j] += ssum[sub + stride][j];
      if (j == 0) ssum[sub][J] += ssum[sub + stride][J];
    }
    __syncthreads();
  }
}

// Level 1: one workgroup per group of at most kRelaxGroup consecutive chunks
// of one row; writes the group's FP64 record.
template <int J>
__global__ __launch_bounds__(256) void k_relaxed_group(const CItem* __restrict__ items, const float* __restrict__ incr,
                                                       double* __restrict__ part) {
  __shared__ double ssum[256 / J][J + 1];
  const CItem it = items[blockIdx.x];
  sum_records<J>(incr + it.in_off * (J + 1), it.count, ssum);
  const int t = threadIdx.x;
  if (t <= J) part[it.out_off * (J + 1) + t] = ssum[0][t];
}

// Level 2: one workgroup per long row, over its groups' records.  a_H (the
// row after its head) is in A(m); the row becomes
//     a_H + omega ((rho^(L - head) - 1) a_H + sum),
//     omega = min(1, 1 / (lr sum ||g||^2)).
template <int J>
__global__ __launch_bounds__(256) void k_relaxed_merge(const CItem* __restrict__ items, const double* __restrict__ part,
                                                       float* __restrict__ Am, double lr, double rho) {
  __shared__ double ssum[256 / J][J + 1];
  const CItem it = items[blockIdx.x];
  sum_records<J>(part + it.in_off * (J + 1), it.count, ssum);
  const int t = threadIdx.x;
  if (t < J) {
    const double lg = lr * ssum[0][J];
    const double omega = lg > 1.0 ? 1.0 / lg : 1.0;
    const double decay = pow(rho, (double)it.out_off);  // out_off: elements after the head
    float* a = Am + (int64_t)it.row * J + t;
    const double aH = (double)*a;
    *a = (float)(aH + omega * ((decay - 1.0) * aH + ssum[0][t]));
  }
}

// One item per 16-lane group: the hardware dispatcher balances the items
// (measured faster than a grid-stride loop, which also costs registers).
unsigned factor_blocks(const void* kernel, int64_t n_items) {
  (void)kernel;
  return (unsigned)std::max<int64_t>(1, (n_items + 15) / 16);
}

template <int N, int J, int R, class T, bool FIB, bool NC = false>
hipError_t factor_launch(const ft_plan* P, int m, const ft_params* p, const Scratch& S, double lr, double lam,
                         hipStream_t s) {
  const ModeMeta& M = P->meta[m];
  const ModeDev& D = P->dev[m];
  const CPtrs<N, T> cp = others<N, T>(p, m);
  NoC<N> nc{};
  if (NC)
    for (int k = 0; k < N - 1; ++k) {
      nc.A[k] = p->A[(m + 1 + k) % N];
      nc.B[k] = p->B[(m + 1 + k) % N];
    }
  const T* Bm = Store<T>::B(p, m);
  const double rho = 1.0 - lr * lam;
  const float flr = (float)lr, c1 = (float)(-lr * lam), gp = (float)(lr / rho);
  if (FIB) {
    KTimer tm(P, FT_K_FIBER_G, s);
    // fiber_batches batches of 16 fibers per 16-lane group, 16 groups per workgroup
    const int64_t per_block = 16 * 16 * fiber_batches<N, R>();
    hipLaunchKernelGGL((k_fiber_g<N, J, R, T>), dim3((unsigned)((M.n_fibers + per_block - 1) / per_block)), dim3(256),
                       0, s, D.fib_idx, M.n_fibers, cp, Bm, S.gfib);
  }
  if constexpr (!NC) {
    if (P->relaxed) {
      // short rows and heads (in place), then the chunks from the rows as their heads left them, then the
      // two merge levels; long rows are read in their dealt order
      const int32_t* fidx = D.fidx ? D.fidx : D.idx;
      const float* fval = D.fval ? D.fval : D.val;
      if (M.n_apply > 0) {
        KTimer tm(P, FT_K_FACTOR_APPLY, s);
        hipLaunchKernelGGL((k_factor_apply<N, J, R, T, FIB>), dim3(factor_blocks(nullptr, M.n_apply)), dim3(256), 0,
                           s, D.apply, M.n_apply, fidx, P->nnz, fval, cp, Bm, p->A[m], nullptr, flr, c1, D.fid,
                           S.gfib, nc, S.maps, D.row_ptr, rho);
      }
      if (M.n_compose > 0) {
        KTimer tm(P, FT_K_FACTOR_COMPOSE, s);
        hipLaunchKernelGGL((k_factor_apply<N, J, R, T, FIB, false, true>), dim3(factor_blocks(nullptr, M.n_compose)),
                           dim3(256), 0, s, D.compose, M.n_compose, fidx, P->nnz, fval, cp, Bm, p->A[m], S.hvec,
                           flr, c1, D.fid, S.gfib, nc, S.maps, D.row_ptr, rho);
      }
      if (M.n_relax > 0) {
        KTimer tm(P, FT_K_COMBINE, s);
        double* part = relax_partials(P, S, m);
        hipLaunchKernelGGL((k_relaxed_group<J>), dim3((unsigned)M.n_relax_groups), dim3(256), 0, s, D.relax,
                           S.maps, part);
        hipLaunchKernelGGL((k_relaxed_merge<J>), dim3((unsigned)M.n_relax), dim3(256), 0, s,
                           D.relax + M.n_relax_groups, part, p->A[m], lr, rho);
      }
      return hipGetLastError();
    }
  }
  if (M.n_compose > 0 && M.n_apply > 0 && P->fused) {
    KTimer tm(P, FT_K_FACTOR_FUSED, s);
    const int64_t ab = (M.n_apply + 15) / 16;
    hipLaunchKernelGGL((k_factor_fused<N, J, R, T, FIB, NC>), dim3((unsigned)(ab + (M.n_compose + 15) / 16)),
                       dim3(256), 0, s, ab, D.apply, M.n_apply, D.compose, M.n_compose, D.idx, P->nnz, D.val, cp, Bm,
                       p->A[m], S.hvec, S.maps, S.map_scale, flr, c1, gp, rho, D.fid, S.gfib, nc);
  } else if (M.n_compose > 0) {
    KTimer tm(P, FT_K_FACTOR_COMPOSE, s);
    hipLaunchKernelGGL((k_factor_compose<N, J, R, T, FIB, NC>),
                       dim3(factor_blocks((const void*)k_factor_compose<N, J, R, T, FIB, NC>, M.n_compose)), dim3(256),
                       0, s, D.compose, M.n_compose, D.idx, P->nnz, D.val, cp, Bm, S.maps, S.map_scale, flr, c1, gp,
                       rho, D.fid, S.gfib, nc);
  }
  if (M.n_apply > 0 && !(M.n_compose > 0 && P->fused)) {
    KTimer tm(P, FT_K_FACTOR_APPLY, s);
    hipLaunchKernelGGL((k_factor_apply<N, J, R, T, FIB, NC>),
                       dim3(factor_blocks((const void*)k_factor_apply<N, J, R, T, FIB, NC>, M.n_apply)), dim3(256), 0,
                       s, D.apply, M.n_apply, D.idx, P->nnz, D.val, cp, Bm, p->A[m], S.hvec, flr, c1, D.fid, S.gfib,
                       nc, S.maps, D.row_ptr, rho);
  }
  for (size_t L = 0; L < M.level_len.size(); ++L) {
    KTimer tm(P, FT_K_COMBINE, s);
    const int64_t nc = M.level_ncomp[L], nf = M.level_len[L] - nc;
    if (nc > 0)
      hipLaunchKernelGGL((k_combine<J>), dim3((unsigned)nc), dim3(256), 0, s, D.levels + M.level_off[L], S.maps,
                         S.map_scale);
    if (nf > 0)
      hipLaunchKernelGGL((k_combine_final<J>), dim3((unsigned)((nf + 15) / 16)), dim3(256), 0, s,
                         D.levels + M.level_off[L] + nc, nf, S.maps, S.map_scale, S.hvec, p->A[m]);
  }
  return hipGetLastError();
}

template <int N, int J, int R, class T>
hipError_t factor_impl(const ft_plan* P, int m, const ft_params* p, const Scratch& S, double lr, double lam,
                       hipStream_t s) {
  if (P->no_c_cache) {
    if constexpr (N == 3 && J == 16 && R == 16 && std::is_same<T, float>::value)
      return factor_launch<N, J, R, T, false, true>(P, m, p, S, lr, lam, s);
    else
      return hipErrorInvalidValue;  // rejected at plan creation and in the parameter checks
  }
  return P->meta[m].use_fiber ? factor_launch<N, J, R, T, true>(P, m, p, S, lr, lam, s)
                              : factor_launch<N, J, R, T, false>(P, m, p, S, lr, lam, s);
}

}  // namespace

int max_fanin(int J) { return J <= 8 ? combine_fanin<8>() : J <= 16 ? combine_fanin<16>() : combine_fanin<32>(); }

hipError_t launch_factor(const ft_plan* P, int m, const ft_params* p, const Scratch& S, double lr, double lam,
                         hipStream_t s) {
#define X(n, j, r)                                                                             \
  case key(n, j, r):                                                                           \
    return bf16(p) ? factor_impl<n, j, r, uint16_t>(P, m, p, S, lr, lam, s)                   \
                   : factor_impl<n, j, r, float>(P, m, p, S, lr, lam, s);
  FT_DISPATCH()
#undef X
}

}  // namespace ft
