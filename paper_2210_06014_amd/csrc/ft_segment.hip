// Segment passes: core gradient, loss, forward, gradient, predict.
#include <mutex>

#include "ft_device.h"

namespace ft {
namespace {

// ---------------------------------------------------------------------------
// Segment passes (core gradient, loss, forward, gradient).  A wavefront takes
// segments gw, gw + nw, ... (a fixed assignment), R/4 lanes per element.

// groups of P elements per trip: fewer at high order, where each element
// holds N - 1 indices in registers
template <int N>
constexpr int trip_unroll() {
  return N > 4 ? 2 : 4;
}

// Values per lane in the segment passes: one 16-byte load of a C row, 4 FP32
// or 8 BF16 values, so a row takes R/4 (FP32) or R/8 (BF16) lanes.
template <class T>
constexpr int vpl() {
  return 16 / (int)sizeof(T);
}

__device__ __forceinline__ void load16(const float* p, float (&o)[4]) {
  const floatx4 u = *reinterpret_cast<const floatx4*>(p);
#pragma unroll
  for (int c = 0; c < 4; ++c) o[c] = u[c];
}
__device__ __forceinline__ void load16(const uint16_t* p, float (&o)[8]) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    o[2 * c] = __uint_as_float(w[c] << 16);
    o[2 * c + 1] = __uint_as_float(w[c] & 0xFFFF0000u);
  }
}

// a 16-byte slice as loaded, widened to its 4 FP32 or 8 BF16 values
template <class T>
__device__ __forceinline__ void widen(const uint4& u, float (&o)[vpl<T>()]) {
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int c = 0; c < 4; ++c) o[c] = __uint_as_float(w[c]);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      o[2 * c] = __uint_as_float(w[c] << 16);
      o[2 * c + 1] = __uint_as_float(w[c] & 0xFFFF0000u);
    }
  }
}

// prod over the gathered 16-byte slices (lane q of the element) of its C
// rows, in table order; zero for an invalid slot.  Invalid slots carry index
// 0 (a valid row), so the loads need no branch and are all in flight together.
template <int N, int R, class T>
__device__ __forceinline__ void gather_slices(const CPtrs<N, T>& cp, const int32_t (&ik)[N > 1 ? N - 1 : 1], bool vld,
                                              int q, float (&w)[vpl<T>()]) {
  constexpr int V = vpl<T>();
  const uint32_t qb = (uint32_t)(16 * q);
  load16(reinterpret_cast<const T*>(reinterpret_cast<const char*>(cp.p[0]) +
                                    ((uint32_t)ik[0] * (uint32_t)(R * sizeof(T)) + qb)),
         w);
#pragma unroll
  for (int k = 1; k < N - 1; ++k) {
    float t[V];
    load16(reinterpret_cast<const T*>(reinterpret_cast<const char*>(cp.p[k]) +
                                      ((uint32_t)ik[k] * (uint32_t)(R * sizeof(T)) + qb)),
           t);
#pragma unroll
    for (int c = 0; c < V; ++c) w[c] *= t[c];
  }
#pragma unroll
  for (int c = 0; c < V; ++c) w[c] = vld ? w[c] : 0.f;
}

// Indices and values of one trip: trip_unroll groups of P elements of a
// segment from position t0.  Each element is loaded once, by lane
// (element - t0) % 64, and handed to the R/4 lanes that gather for it by a
// cross-lane permute (the LDS crossbar), so that an index load carries 64
// distinct addresses: the address units, which bound these passes, see a
// quarter of the index loads.  Positions past the end are clamped to the
// segment's last element (a valid address), so the loads need no branch.
// A trip of fewer than 32 elements (R = 32 at high orders) would waste most
// of such loads, so there each lane loads its own elements' indices.
template <int N, int P>
struct Trip {
  static constexpr int U = trip_unroll<N>();
  static constexpr bool PERMUTE = U * P >= 32;
  static constexpr int NL = PERMUTE ? (U * P + 63) / 64 : U;  // element loads per lane
  int32_t ik[NL][N > 1 ? N - 1 : 1];
  float xv[NL];
};

template <int N, int P, bool PERM>
__device__ __forceinline__ void load_trip(Trip<N, P>& L, const Seg& S, int t0, int lane,
                                          const int32_t* __restrict__ idx, int64_t nnz, const float* __restrict__ xs,
                                          const int32_t* __restrict__ perm) {
  const int last = max(S.len - 1, 0);
  const int slot = lane / (64 / P);
#pragma unroll
  for (int h = 0; h < Trip<N, P>::NL; ++h) {
    const uint32_t o = (uint32_t)min(Trip<N, P>::PERMUTE ? t0 + 64 * h + lane : t0 + h * P + slot, last);
#pragma unroll
    for (int k = 0; k < N - 1; ++k) L.ik[h][k] = (idx + (int64_t)k * nnz + S.start)[o];
    L.xv[h] = PERM ? xs[(perm + S.start)[o]] : (xs + S.start)[o];
  }
}

// indices and value of element u P + slot of a trip, from the lane that loaded it
template <int N, int P, int u>
__device__ __forceinline__ void trip_elem(const Trip<N, P>& L, int slot, int32_t (&ik)[N > 1 ? N - 1 : 1],
                                          float& xv) {
  if constexpr (Trip<N, P>::PERMUTE) {
    constexpr int h = (u * P) / 64;
    const int src = (u * P + slot) & 63;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) ik[k] = __shfl(L.ik[h][k], src);
    xv = __shfl(L.xv[h], src);
  } else {
#pragma unroll
    for (int k = 0; k < N - 1; ++k) ik[k] = L.ik[u][k];
    xv = L.xv[u];
  }
}

// A wavefront walks its segments gw, gw + nw, ... trip by trip.  While the
// gathers of one trip are in flight it already loads the indices of the next
// trip (the first trip of its next segment at a segment's end, whose
// descriptor was read one segment ahead), so that every trip costs one memory
// round trip instead of two.  A segment of length 0 stands in past the last.

// MODE 0: s = sum e w (core gradient); MODE 1: t = sum -e w (gradient of 1/2 sum e^2);
// MODE 2: t = sum delta w with delta from the caller (input order, via perm).
template <int N, int J, int R, int MODE, class T>
__global__ __launch_bounds__(256) void k_segsum(const Seg* __restrict__ segs, int64_t nseg,
                                                const int32_t* __restrict__ idx, int64_t nnz,
                                                const float* __restrict__ val, CPtrs<N, T> cp,
                                                const T* __restrict__ Cm, const T* __restrict__ Am,
                                                const float* __restrict__ up, const int32_t* __restrict__ perm,
                                                float* __restrict__ partials, float* __restrict__ tseg) {
  constexpr int V = vpl<T>();
  constexpr int QL = R / V;
  constexpr int P = 64 / QL;
  constexpr int GJ = (J + P - 1) / P;
  constexpr int U = trip_unroll<N>();
  __shared__ float red[4][J * R];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slot = lane / QL, q = lane % QL;
  const int64_t nw = (int64_t)gridDim.x * 4;
  const float* xs = MODE == 2 ? up : val;
  float Gp[GJ][V];
#pragma unroll
  for (int u = 0; u < GJ; ++u)
#pragma unroll
    for (int c = 0; c < V; ++c) Gp[u][c] = 0.f;
  // C(m) slice and A(m) entries of a segment's row
  auto row_loads = [&](const Seg& X, float (&cr)[V], float (&ar)[GJ]) {
    if (MODE != 2) load16(Cm + (int64_t)X.row * R + V * q, cr);
#pragma unroll
    for (int u = 0; u < GJ; ++u) {
      const int j = slot + P * u;
      ar[u] = j < J ? to_f(Am[(int64_t)X.row * J + j]) : 0.f;
    }
  };
  int64_t sg = (int64_t)blockIdx.x * 4 + wave;
  if (sg < nseg) {
    const Seg none{0, 0, 0};
    Seg S = segs[sg];
    Seg Sq = sg + nw < nseg ? segs[sg + nw] : none;
    float crow[V];
#pragma unroll
    for (int c = 0; c < V; ++c) crow[c] = 0.f;
    float arow[GJ];
    row_loads(S, crow, arow);
    Trip<N, P> cur;
    load_trip<N, P, MODE == 2>(cur, S, 0, lane, idx, nnz, xs, perm);
    float acc[V];
#pragma unroll
    for (int c = 0; c < V; ++c) acc[c] = 0.f;
    int t0 = 0;
    for (;;) {
      int32_t ik[U][N > 1 ? N - 1 : 1];
      float xv[U];
      bool vl[U];
      static_for<0, U>([&](auto UU) {
        constexpr int u = decltype(UU)::value;
        trip_elem<N, P, u>(cur, slot, ik[u], xv[u]);
        vl[u] = t0 + u * P + slot < S.len;
      });
      float w[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u) gather_slices<N, R, T>(cp, ik[u], vl[u], q, w[u]);
      const bool seg_end = t0 + P * U >= S.len;
      const Seg& Sn = seg_end ? Sq : S;
      Trip<N, P> nxt;
      load_trip<N, P, MODE == 2>(nxt, Sn, seg_end ? 0 : t0 + P * U, lane, idx, nnz, xs, perm);
      float crow_n[V], arow_n[GJ];
#pragma unroll
      for (int c = 0; c < V; ++c) crow_n[c] = crow[c];
#pragma unroll
      for (int u = 0; u < GJ; ++u) arow_n[u] = arow[u];
      if (seg_end) row_loads(Sq, crow_n, arow_n);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float d;
        if (MODE == 2) {
          d = vl[u] ? xv[u] : 0.f;
        } else {
          float xh = crow[0] * w[u][0];
#pragma unroll
          for (int c = 1; c < V; ++c) xh = fmaf(crow[c], w[u][c], xh);
          xh = group_sum<QL>(xh);
          d = vl[u] ? (MODE == 0 ? xv[u] - xh : xh - xv[u]) : 0.f;
        }
#pragma unroll
        for (int c = 0; c < V; ++c) acc[c] = fmaf(d, w[u][c], acc[c]);
      }
      if (seg_end) {
#pragma unroll
        for (int off = QL; off < 64; off <<= 1)
#pragma unroll
          for (int c = 0; c < V; ++c) acc[c] += __shfl_xor(acc[c], off);
        if (tseg && slot == 0)
#pragma unroll
          for (int c = 0; c < V; ++c) tseg[sg * R + V * q + c] = acc[c];
#pragma unroll
        for (int u = 0; u < GJ; ++u) {
          const int j = slot + P * u;
          if (j < J)
#pragma unroll
            for (int c = 0; c < V; ++c) Gp[u][c] = fmaf(arow[u], acc[c], Gp[u][c]);
        }
        sg += nw;
        if (sg >= nseg) break;
        S = Sq;
        Sq = sg + nw < nseg ? segs[sg + nw] : none;
#pragma unroll
        for (int c = 0; c < V; ++c) {
          crow[c] = crow_n[c];
          acc[c] = 0.f;
        }
#pragma unroll
        for (int u = 0; u < GJ; ++u) arow[u] = arow_n[u];
        t0 = 0;
      } else {
        t0 += P * U;
      }
      cur = nxt;
    }
  }
#pragma unroll
  for (int u = 0; u < GJ; ++u) {
    const int j = slot + P * u;
    if (j < J)
#pragma unroll
      for (int c = 0; c < V; ++c) red[wave][j * R + V * q + c] = Gp[u][c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < J * R; e += 256)
    partials[(int64_t)blockIdx.x * J * R + e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// ---------------------------------------------------------------------------
// Segment passes with the C row of the first index column reused along runs.
// Within a row of mode m the elements are sorted by the index of mode m + 1
// (column 0 of idx), so consecutive elements repeat it in runs (at order 3 the
// fibers of the third mode).  Here the P slots of a wavefront (R/V lanes
// each) take contiguous pieces of a segment, so that a run stays within a
// slot, and a slot gathers the column-0 row only where that index changes:
// per element it gathers the rows of the other columns, per run one more.
// With u = C(m)[row] * C(m+1)[j] formed once per run,
//     xhat = u . prod_{k >= 1} C[i_k]                        (per element)
//     s = sum_x e_x w_x = sum_runs C(m+1)[j] * t_run,  t_run = sum_{x in run} e_x prod_{k >= 1} C[i_k].
// MODE 0, 1, 2 as in k_segsum; MODE 3: loss (FP64 sum of e^2) and, with out,
// xhat stored at the element's input position.  The walk, the partials and
// the fixed summation order are otherwise those of k_segsum: a wavefront
// takes segments gw, gw + nw, ..., and each trip of U steps loads the indices
// of the next trip (across segment boundaries) while its gathers are in
// flight.
template <int N, int J, int R, int MODE, class T>
__global__ __launch_bounds__(256) void k_segrun(const Seg* __restrict__ segs, int64_t nseg,
                                                const int32_t* __restrict__ idx, int64_t nnz,
                                                const float* __restrict__ val, CPtrs<N, T> cp,
                                                const T* __restrict__ Cm, const T* __restrict__ Am,
                                                const float* __restrict__ up, const int32_t* __restrict__ perm,
                                                float* __restrict__ partials, float* __restrict__ tseg,
                                                double* __restrict__ dpart, float* __restrict__ out) {
  static_assert(N >= 3, "run reuse needs a column besides the first");
  constexpr int V = vpl<T>();
  constexpr int QL = R / V;               // lanes per element
  constexpr int P = 64 / QL;              // slots per wavefront
  constexpr int GJ = (J + P - 1) / P;
  constexpr int U = N > 4 ? 2 : 4;        // steps per trip
  constexpr int NL = (U + QL - 1) / QL;   // element loads per lane per trip
  constexpr int NI = N - 1;
  constexpr bool LOSS = MODE == 3;
  constexpr bool PERM = MODE == 2;
  __shared__ float red[LOSS ? 1 : 4][LOSS ? 1 : J * R];
  __shared__ double dred[4];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slot = lane / QL, q = lane % QL;
  const int64_t nw = (int64_t)gridDim.x * 4;
  const float* xs = PERM ? up : val;
  float Gp[LOSS ? 1 : GJ][V];
#pragma unroll
  for (int u = 0; u < (LOSS ? 1 : GJ); ++u)
#pragma unroll
    for (int c = 0; c < V; ++c) Gp[u][c] = 0.f;
  double sse = 0.0;
  // loads of one trip: lane q of a slot loads the slot's elements q, q + QL, ... of the trip
  struct Ld {
    int32_t ik[NL][NI];
    float xv[NL];
  };
  auto load_trip = [&](Ld& L, const Seg& X, int k0) {
    const int Ls = (X.len + P - 1) / P;
    const int last = max(X.len - 1, 0);
#pragma unroll
    for (int h = 0; h < NL; ++h) {
      const uint32_t o = (uint32_t)min(slot * Ls + k0 + q + QL * h, last);
#pragma unroll
      for (int k = 0; k < NI; ++k) L.ik[h][k] = (idx + (int64_t)k * nnz + X.start)[o];
      L.xv[h] = PERM ? xs[(perm + X.start)[o]] : (xs + X.start)[o];
    }
  };
  auto row_loads = [&](const Seg& X, float (&cr)[V], float (&ar)[LOSS ? 1 : GJ]) {
    if (MODE != 2) load16(Cm + (int64_t)X.row * R + V * q, cr);
    if constexpr (!LOSS) {
#pragma unroll
      for (int u = 0; u < GJ; ++u) {
        const int j = slot + P * u;
        ar[u] = j < J ? to_f(Am[(int64_t)X.row * J + j]) : 0.f;
      }
    }
  };
  int64_t sg = (int64_t)blockIdx.x * 4 + wave;
  if (sg < nseg) {
    const Seg none{0, 0, 0};
    Seg S = segs[sg];
    Seg Sq = sg + nw < nseg ? segs[sg + nw] : none;
    float crow[V], arow[LOSS ? 1 : GJ];
#pragma unroll
    for (int c = 0; c < V; ++c) crow[c] = 0.f;
    row_loads(S, crow, arow);
    Ld cur;
    load_trip(cur, S, 0);
    int Ls = (S.len + P - 1) / P;
    int b = slot * Ls, e = min(S.len, b + Ls);
    // run state of this slot: the column-0 index and row of the current run,
    // u = crow * c1, the run's partial sum t, the segment's sum s
    int32_t jprev = -1;
    float c1[V], uu[V], t[V], s[V];
#pragma unroll
    for (int c = 0; c < V; ++c) c1[c] = uu[c] = t[c] = s[c] = 0.f;
    int k0 = 0;
    for (;;) {
      int32_t ik[U][NI];
      float xv[U];
      bool vl[U], nr[U];
      static_for<0, U>([&](auto UU) {
        constexpr int u = decltype(UU)::value;
        constexpr int h = u / QL;
        const int src = slot * QL + (u % QL);
#pragma unroll
        for (int k = 0; k < NI; ++k) ik[u][k] = QL > 1 ? __shfl(cur.ik[h][k], src) : cur.ik[h][k];
        xv[u] = QL > 1 ? __shfl(cur.xv[h], src) : cur.xv[h];
        vl[u] = b + k0 + u < e;
      });
      // a step starts a run where its column-0 index differs from the step before
      nr[0] = vl[0] && ik[0][0] != jprev;
#pragma unroll
      for (int u = 1; u < U; ++u) nr[u] = vl[u] && ik[u][0] != ik[u - 1][0];
      // gathers: the rows of columns 1.. for every step, the column-0 row where a run starts
      // slices are kept as loaded (four registers, FP32 or BF16) and widened
      // where used; at order 4 and up the per-element product is formed here
      constexpr bool PROD = NI > 2;
      uint4 w2r[U], cnr[U];
      float w2p[PROD ? U : 1][PROD ? V : 1];
      const uint32_t qb = (uint32_t)(16 * q);
      auto slice = [&](int k, int32_t i) {
        return *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(cp.p[k]) +
                                               ((uint32_t)i * (uint32_t)(R * sizeof(T)) + qb));
      };
#pragma unroll
      for (int u = 0; u < U; ++u) {
        w2r[u] = slice(1, ik[u][1]);
        if constexpr (PROD) {
          widen<T>(w2r[u], w2p[u]);
#pragma unroll
          for (int k = 2; k < NI; ++k) {
            float tk[V];
            widen<T>(slice(k, ik[u][k]), tk);
#pragma unroll
            for (int c = 0; c < V; ++c) w2p[u][c] *= tk[c];
          }
        }
        cnr[u] = make_uint4(0u, 0u, 0u, 0u);
        if (nr[u]) cnr[u] = slice(0, ik[u][0]);
      }
      // the next trip's indices (the next segment's first trip at a segment's end)
      const bool seg_end = k0 + U >= Ls;
      const Seg& Sn = seg_end ? Sq : S;
      Ld nxt;
      load_trip(nxt, Sn, seg_end ? 0 : k0 + U);
      float crow_n[V], arow_n[LOSS ? 1 : GJ];
#pragma unroll
      for (int c = 0; c < V; ++c) crow_n[c] = crow[c];
#pragma unroll
      for (int u = 0; u < (LOSS ? 1 : GJ); ++u) arow_n[u] = arow[u];
      if (seg_end) row_loads(Sq, crow_n, arow_n);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float w2[V];
        if constexpr (PROD) {
#pragma unroll
          for (int c = 0; c < V; ++c) w2[c] = w2p[u][c];
        } else {
          widen<T>(w2r[u], w2);
        }
        if (nr[u]) {
          // close the previous run: s += C(m+1)[j] * t
          float cn[V];
          widen<T>(cnr[u], cn);
#pragma unroll
          for (int c = 0; c < V; ++c) {
            s[c] = fmaf(c1[c], t[c], s[c]);
            t[c] = 0.f;
            c1[c] = cn[c];
            uu[c] = crow[c] * c1[c];
          }
        }
        if (vl[u]) jprev = ik[u][0];
        float d;
        if constexpr (MODE == 2) {
          d = vl[u] ? xv[u] : 0.f;
        } else {
          float xh = uu[0] * w2[0];
#pragma unroll
          for (int c = 1; c < V; ++c) xh = fmaf(uu[c], w2[c], xh);
          xh = group_sum<QL>(xh);
          if constexpr (LOSS) {
            if (vl[u] && q == 0) {
              const float er = xv[u] - xh;
              sse += (double)er * (double)er;
              if (out) out[perm[S.start + (b + k0 + u)]] = xh;
            }
            d = 0.f;
          } else {
            d = vl[u] ? (MODE == 0 ? xv[u] - xh : xh - xv[u]) : 0.f;
          }
        }
        if constexpr (!LOSS) {
#pragma unroll
          for (int c = 0; c < V; ++c) t[c] = fmaf(d, w2[c], t[c]);
        }
      }
      if (seg_end) {
        if constexpr (!LOSS) {
#pragma unroll
          for (int c = 0; c < V; ++c) s[c] = fmaf(c1[c], t[c], s[c]);
#pragma unroll
          for (int off = QL; off < 64; off <<= 1)
#pragma unroll
            for (int c = 0; c < V; ++c) s[c] += __shfl_xor(s[c], off);
          if (tseg && slot == 0)
#pragma unroll
            for (int c = 0; c < V; ++c) tseg[sg * R + V * q + c] = s[c];
#pragma unroll
          for (int u = 0; u < GJ; ++u) {
            const int j = slot + P * u;
            if (j < J)
#pragma unroll
              for (int c = 0; c < V; ++c) Gp[u][c] = fmaf(arow[u], s[c], Gp[u][c]);
          }
        }
        sg += nw;
        if (sg >= nseg) break;
        S = Sq;
        Sq = sg + nw < nseg ? segs[sg + nw] : none;
        Ls = (S.len + P - 1) / P;
        b = slot * Ls;
        e = min(S.len, b + Ls);
        jprev = -1;
#pragma unroll
        for (int c = 0; c < V; ++c) {
          crow[c] = crow_n[c];
          c1[c] = uu[c] = t[c] = s[c] = 0.f;
        }
#pragma unroll
        for (int u = 0; u < (LOSS ? 1 : GJ); ++u) arow[u] = arow_n[u];
        k0 = 0;
      } else {
        k0 += U;
      }
      cur = nxt;
    }
  }
  if constexpr (LOSS) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) sse += __shfl_xor(sse, off);
    if (lane == 0) dred[wave] = sse;
    __syncthreads();
    if (threadIdx.x == 0 && dpart) dpart[blockIdx.x] = ((dred[0] + dred[1]) + dred[2]) + dred[3];
  } else {
#pragma unroll
    for (int u = 0; u < GJ; ++u) {
      const int j = slot + P * u;
      if (j < J)
#pragma unroll
        for (int c = 0; c < V; ++c) red[wave][j * R + V * q + c] = Gp[u][c];
    }
    __syncthreads();
    for (int x = threadIdx.x; x < J * R; x += 256)
      partials[(int64_t)blockIdx.x * J * R + x] = ((red[0][x] + red[1][x]) + red[2][x]) + red[3][x];
  }
}

// Core gradient without the C cache (the Table 5 comparison; N = 3,
// J = R = 16): one segment per 16-lane group.  Lane r forms C(n)[i, r] of the
// other modes from their A rows, C(m)[row, r] once per segment, then
// s_r = sum_x e_x w_r and G[:, r] += a_row s_r.  The sixteen groups' partials
// of a workgroup are summed in a fixed order.
template <int N>
__global__ __launch_bounds__(256) void k_core_nc(const Seg* __restrict__ segs, int64_t nseg,
                                                 const int32_t* __restrict__ idx, int64_t nnz,
                                                 const float* __restrict__ val, NoC<N> nc,
                                                 const float* __restrict__ Am, const float* __restrict__ Bm,
                                                 float* __restrict__ partials) {
  constexpr int J = 16, R = 16;
  __shared__ float red[16][J * R];
  const int l = threadIdx.x & 15, grp = threadIdx.x >> 4;
  float Bc[N - 1][16];
  load_nc_cols<N>(nc, l, Bc);
  float Bmc[16], Gc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    Bmc[j] = Bm[j * R + l];
    Gc[j] = 0.f;
  }
  const int64_t ng = (int64_t)gridDim.x * 16;
  for (int64_t sg = (int64_t)blockIdx.x * 16 + grp; sg < nseg; sg += ng) {
    const Seg S = segs[sg];
    const float arow = Am[(int64_t)S.row * J + l];
    float crow = 0.f;
    dot_bcast16(crow, arow, Bmc);  // C(m)[row, l]
    float sacc = 0.f;
    for (int t0 = 0; t0 < S.len; t0 += 16) {
      const int64_t p = S.start + min(t0 + l, S.len - 1);
      const float xv = val[p];
      int ix[N - 1];
#pragma unroll
      for (int k = 0; k < N - 1; ++k) ix[k] = idx[(int64_t)k * nnz + p];
      float w[16][1];
      gather_w_nc<N>(nc, Bc, ix, l, t0, S.len, w);
      static_for<0, 16>([&](auto SS) {
        constexpr int s = decltype(SS)::value;
        const float xh = group_sum<16>(crow * w[s][0]);
        const float e = bcast16<s>(xv) - xh;
        sacc = fmaf(e, w[s][0], sacc);  // w = 0 past the end of the segment
      });
    }
    axpy_bcast16(Gc, arow, sacc);  // G[j][l] += a_j s_l
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) red[grp][j * R + l] = Gc[j];
  __syncthreads();
  for (int e = threadIdx.x; e < J * R; e += 256) {
    float acc = 0.f;
#pragma unroll
    for (int g = 0; g < 16; ++g) acc += red[g][e];
    partials[(int64_t)blockIdx.x * J * R + e] = acc;
  }
}

// Sum of the workgroup partials in a fixed order, in two stages: first every
// block of kFold consecutive partials (many workgroups), then the blocks.
constexpr int kFold = 32;

__global__ __launch_bounds__(256) void k_fold_partials(const float* __restrict__ partials, int nparts, int JR,
                                                       float* __restrict__ folded) {
  const int b0 = blockIdx.x * kFold;
  const int nb = min(kFold, nparts - b0);
  for (int e = threadIdx.x; e < JR; e += blockDim.x) {
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += partials[(int64_t)(b0 + b) * JR + e];
    folded[(int64_t)blockIdx.x * JR + e] = s;
  }
}

// Final sum; optionally the core step B <- B + lr (G / |Omega| - lam B) (Algorithm 5).
__global__ __launch_bounds__(256) void k_reduce_update(const float* __restrict__ folded, int nfold, int JR,
                                                       float* __restrict__ Bm, float* __restrict__ Gout, float lr,
                                                       float lam, float inv_nnz, int update) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= JR) return;
  float s = 0.f;
  for (int b = 0; b < nfold; ++b) s += folded[(int64_t)b * JR + e];
  if (Gout) Gout[e] = s;
  if (update) {
    const float b = Bm[e];
    Bm[e] = b + lr * (s * inv_nnz - lam * b);
  }
}

// dA(m)[i, j] = sum_r B(m)[j, r] t_i[r], t_i = sum of the row's segment sums.
template <int J, int R, class T>
__global__ __launch_bounds__(256) void k_grad_rows(const int64_t* __restrict__ seg_ptr, const float* __restrict__ tseg,
                                                   const T* __restrict__ Bm, float* __restrict__ gA, int64_t I) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= I * J) return;
  const int64_t i = e / J;
  const int j = (int)(e % J);
  float t[R];
#pragma unroll
  for (int r = 0; r < R; ++r) t[r] = 0.f;
  for (int64_t sg = seg_ptr[i]; sg < seg_ptr[i + 1]; ++sg)
#pragma unroll
    for (int r = 0; r < R; ++r) t[r] += tseg[sg * R + r];
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < R; ++r) s = fmaf(to_f(Bm[j * R + r]), t[r], s);
  gA[e] = s;
}

// Loss: per-element e^2 summed in FP64 (and, with out != nullptr, xhat stored
// at the element's input position).
template <int N, int R, class T>
__global__ __launch_bounds__(256) void k_loss(const Seg* __restrict__ segs, int64_t nseg,
                                              const int32_t* __restrict__ idx, int64_t nnz,
                                              const float* __restrict__ val, CPtrs<N, T> cp,
                                              const T* __restrict__ Cm, double* __restrict__ dpart,
                                              const int32_t* __restrict__ perm, float* __restrict__ out) {
  constexpr int V = vpl<T>();
  constexpr int QL = R / V;
  constexpr int P = 64 / QL;
  constexpr int U = trip_unroll<N>();
  __shared__ double red[4];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slot = lane / QL, q = lane % QL;
  const int64_t nw = (int64_t)gridDim.x * 4;
  double sse = 0.0;
  int64_t sg = (int64_t)blockIdx.x * 4 + wave;
  if (sg < nseg) {
    const Seg none{0, 0, 0};
    Seg S = segs[sg];
    Seg Sq = sg + nw < nseg ? segs[sg + nw] : none;
    float crow[V];
    load16(Cm + (int64_t)S.row * R + V * q, crow);
    Trip<N, P> cur;
    load_trip<N, P, false>(cur, S, 0, lane, idx, nnz, val, nullptr);
    int t0 = 0;
    for (;;) {
      int32_t ik[U][N > 1 ? N - 1 : 1];
      float xv[U];
      bool vl[U];
      static_for<0, U>([&](auto UU) {
        constexpr int u = decltype(UU)::value;
        trip_elem<N, P, u>(cur, slot, ik[u], xv[u]);
        vl[u] = t0 + u * P + slot < S.len;
      });
      float w[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u) gather_slices<N, R, T>(cp, ik[u], vl[u], q, w[u]);
      const bool seg_end = t0 + P * U >= S.len;
      const Seg& Sn = seg_end ? Sq : S;
      Trip<N, P> nxt;
      load_trip<N, P, false>(nxt, Sn, seg_end ? 0 : t0 + P * U, lane, idx, nnz, val, nullptr);
      float crow_n[V];
      if (seg_end) {
        load16(Cm + (int64_t)Sq.row * R + V * q, crow_n);
      } else {
#pragma unroll
        for (int c = 0; c < V; ++c) crow_n[c] = crow[c];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float xh = crow[0] * w[u][0];
#pragma unroll
        for (int c = 1; c < V; ++c) xh = fmaf(crow[c], w[u][c], xh);
        xh = group_sum<QL>(xh);
        if (vl[u] && q == 0) {
          const float e = xv[u] - xh;
          sse += (double)e * (double)e;
          if (out) out[perm[S.start + (t0 + u * P + slot)]] = xh;
        }
      }
      if (seg_end) {
        sg += nw;
        if (sg >= nseg) break;
        S = Sq;
        Sq = sg + nw < nseg ? segs[sg + nw] : none;
        t0 = 0;
      } else {
        t0 += P * U;
      }
#pragma unroll
      for (int c = 0; c < V; ++c) crow[c] = crow_n[c];
      cur = nxt;
    }
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) sse += __shfl_xor(sse, off);
  if (lane == 0) red[wave] = sse;
  __syncthreads();
  if (threadIdx.x == 0 && dpart) dpart[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// FP64 sum of squares of a matrix, one partial per workgroup.
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ X, int64_t n, double* __restrict__ dpart) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    const double x = X[k];
    s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) dpart[blockIdx.x] = red[0];
}

constexpr int kSumsqBlocks = 256;

// Fixed-order FP64 sums of the partials (strided per thread, then a tree).
__global__ __launch_bounds__(256) void k_loss_finish(const double* __restrict__ dpart, int n_sse,
                                                     const double* __restrict__ rpart, int n_a, int n_b, double nnz,
                                                     double lam_a, double lam_b, double* __restrict__ out4) {
  __shared__ double red[3][256];
  const int t = threadIdx.x;
  double sse = 0.0, ra = 0.0, rb = 0.0;
  for (int k = t; k < n_sse; k += 256) sse += dpart[k];
  for (int k = t; k < n_a; k += 256) ra += rpart[k];
  for (int k = t; k < n_b; k += 256) rb += rpart[n_a + k];
  red[0][t] = sse;
  red[1][t] = ra;
  red[2][t] = rb;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
      for (int c = 0; c < 3; ++c) red[c][t] += red[c][t + h];
    __syncthreads();
  }
  if (t == 0) {
    out4[0] = red[0][0];
    out4[1] = nnz > 0 ? sqrt(red[0][0] / nnz) : 0.0;
    out4[2] = lam_a * red[1][0];
    out4[3] = lam_b * red[2][0];
  }
}

// Predictions for query coordinates (structure of arrays [N][q]).
template <int N, int R, class T>
__global__ __launch_bounds__(256) void k_predict(const int32_t* __restrict__ coords, int64_t q,
                                                 CPtrs<N + 1, T> cp, float* __restrict__ out) {
  constexpr int QL = R / 4;
  const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t x = tid / QL;
  const int qq = (int)(tid % QL);
  const bool vld = x < q;
  floatx4 w = {1.f, 1.f, 1.f, 1.f};
#pragma unroll
  for (int n = 0; n < N; ++n) {
    const int32_t i = vld ? coords[(int64_t)n * q + x] : 0;
    const floatx4 c = load4(cp.p[n] + (int64_t)i * R + 4 * qq);
    w *= c;
  }
  float s = ((w[0] + w[1]) + w[2]) + w[3];
  s = group_sum<QL>(s);
  if (vld && qq == 0) out[x] = s;
}


hipError_t reduce_partials(const ft_plan* P, const Scratch& S, int nparts, float* Bm, float* Gout, float lr,
                           float lam, float inv, int update, hipStream_t s) {
  KTimer tm(P, FT_K_REDUCE, s);
  const int JR = P->J * P->R;
  const int nfold = (nparts + kFold - 1) / kFold;
  float* folded = S.partials + (int64_t)kPartials * JR;
  if (nfold > 0) hipLaunchKernelGGL(k_fold_partials, dim3(nfold), dim3(256), 0, s, S.partials, nparts, JR, folded);
  hipLaunchKernelGGL(k_reduce_update, dim3((JR + 255) / 256), dim3(256), 0, s, folded, nfold, JR, Bm, Gout, lr, lam,
                     inv, update);
  return hipGetLastError();
}

int seg_blocks(const void* kernel, int64_t nseg) {
  int64_t b = (nseg + 3) / 4;
  b = std::min<int64_t>(b, std::min(kPartials, resident_blocks(kernel)));
  if (b < 1) b = 1;
  return (int)b;
}

template <int N, int J, int R, class T>
hipError_t segsum_impl(const ft_plan* P, int m, const ft_params* p, float* partials, int mode, const float* up,
                       float* tseg, hipStream_t s, int* nblocks) {
  const ModeMeta& M = P->meta[m];
  const ModeDev& D = P->dev[m];
  const CPtrs<N, T> cp = others<N, T>(p, m);
  const T* Cm = Store<T>::C(p, m);
  const T* Am = Store<T>::A(p, m);
  // modes 0 and 1 (the core gradient and the gradient of 1/2 sum e^2) launch
  // the same grid, so their sums run in the same order and one is the exact
  // negation of the other
  if constexpr (N >= 3) {
    if (P->run_reuse) {
      const void* kr = mode == 2 ? (const void*)k_segrun<N, J, R, 2, T> : (const void*)k_segrun<N, J, R, 0, T>;
      const int nbr = seg_blocks(kr, M.n_segs);
      *nblocks = nbr;
      KTimer tm(P, FT_K_SEGSUM, s);
      if (mode == 0)
        hipLaunchKernelGGL((k_segrun<N, J, R, 0, T>), dim3(nbr), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz,
                           D.val, cp, Cm, Am, nullptr, nullptr, partials, tseg, nullptr, nullptr);
      else if (mode == 1)
        hipLaunchKernelGGL((k_segrun<N, J, R, 1, T>), dim3(nbr), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz,
                           D.val, cp, Cm, Am, nullptr, nullptr, partials, tseg, nullptr, nullptr);
      else
        hipLaunchKernelGGL((k_segrun<N, J, R, 2, T>), dim3(nbr), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz,
                           D.val, cp, Cm, Am, up, D.perm, partials, tseg, nullptr, nullptr);
      return hipGetLastError();
    }
  }
  const void* kern = mode == 2 ? (const void*)k_segsum<N, J, R, 2, T> : (const void*)k_segsum<N, J, R, 0, T>;
  const int nb = seg_blocks(kern, M.n_segs);
  *nblocks = nb;
  KTimer tm(P, FT_K_SEGSUM, s);
  if (mode == 0)
    hipLaunchKernelGGL((k_segsum<N, J, R, 0, T>), dim3(nb), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz, D.val,
                       cp, Cm, Am, nullptr, nullptr, partials, tseg);
  else if (mode == 1)
    hipLaunchKernelGGL((k_segsum<N, J, R, 1, T>), dim3(nb), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz, D.val,
                       cp, Cm, Am, nullptr, nullptr, partials, tseg);
  else
    hipLaunchKernelGGL((k_segsum<N, J, R, 2, T>), dim3(nb), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz, D.val,
                       cp, Cm, Am, up, D.perm, partials, tseg);
  return hipGetLastError();
}

// dpart: kPartials FP64 partials of the loss kernel, then 2 N kSumsqBlocks of
// the regularisers.
template <int N, int J, int R, class T>
hipError_t loss_impl(const ft_plan* P, const ft_params* p, double* dpart, double lam_a, double lam_b, double* out4,
                     float* xout, hipStream_t s) {
  // the loss is a sum over all elements: any mode's CSR serves; with run
  // reuse the plan picks the mode with the longest runs
  const int lm = P->run_reuse ? P->loss_mode : 0;
  const ModeMeta& M = P->meta[lm];
  const ModeDev& D = P->dev[lm];
  const CPtrs<N, T> cp = others<N, T>(p, lm);
  int nb = 0;
  if constexpr (N >= 3) {
    if (P->run_reuse) {
      nb = seg_blocks((const void*)k_segrun<N, J, R, 3, T>, M.n_segs);
      KTimer tm(P, FT_K_LOSS, s);
      hipLaunchKernelGGL((k_segrun<N, J, R, 3, T>), dim3(nb), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz,
                         D.val, cp, Store<T>::C(p, lm), nullptr, nullptr, D.perm, nullptr, nullptr,
                         out4 ? dpart : nullptr, xout);
    }
  }
  if (nb == 0) {
    nb = seg_blocks((const void*)k_loss<N, R, T>, M.n_segs);
    KTimer tm(P, FT_K_LOSS, s);
    hipLaunchKernelGGL((k_loss<N, R, T>), dim3(nb), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz, D.val, cp,
                       Store<T>::C(p, lm), out4 ? dpart : nullptr, D.perm, xout);
  }
  if (!out4) return hipGetLastError();
  // the regularisers of Eq. (6) are taken on the FP32 masters
  KTimer tm(P, FT_K_REDUCE, s);
  double* rpart = dpart + kPartials;
  for (int n = 0; n < N; ++n)
    hipLaunchKernelGGL(k_sumsq, dim3(kSumsqBlocks), dim3(256), 0, s, p->A[n], P->desc.dims[n] * J,
                       rpart + n * kSumsqBlocks);
  for (int n = 0; n < N; ++n)
    hipLaunchKernelGGL(k_sumsq, dim3(kSumsqBlocks), dim3(256), 0, s, p->B[n], (int64_t)J * R,
                       rpart + (N + n) * kSumsqBlocks);
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, dpart, nb, rpart, N * kSumsqBlocks,
                     N * kSumsqBlocks, (double)P->nnz, lam_a, lam_b, out4);
  return hipGetLastError();
}

template <int N, int R, class T>
hipError_t predict_impl(const ft_params* p, const int32_t* coords, int64_t q, float* out, hipStream_t s) {
  CPtrs<N + 1, T> cp{};
  for (int n = 0; n < N; ++n) cp.p[n] = Store<T>::C(p, n);
  const int64_t threads = q * (R / 4);
  const unsigned nb = (unsigned)((threads + 255) / 256);
  if (nb > 0) hipLaunchKernelGGL((k_predict<N, R, T>), dim3(nb), dim3(256), 0, s, coords, q, cp, out);
  return hipGetLastError();
}

template <int J, int R, class T>
hipError_t grad_rows_impl(const ft_plan* P, int m, const ft_params* p, const float* tseg, float* gA, hipStream_t s) {
  const int64_t I = P->desc.dims[m];
  const unsigned gb = (unsigned)((I * J + 255) / 256);
  if (gb > 0)
    hipLaunchKernelGGL((k_grad_rows<J, R, T>), dim3(gb), dim3(256), 0, s, P->dev[m].seg_ptr, tseg,
                       Store<T>::B(p, m), gA, I);
  return hipGetLastError();
}

}  // namespace

static hipError_t segsum(const ft_plan* P, int m, const ft_params* p, float* partials, int mode, const float* up,
                         float* tseg, hipStream_t s, int* nb) {
#define X(n, j, r)                                                                             \
  case key(n, j, r):                                                                           \
    return bf16(p) ? segsum_impl<n, j, r, uint16_t>(P, m, p, partials, mode, up, tseg, s, nb) \
                   : segsum_impl<n, j, r, float>(P, m, p, partials, mode, up, tseg, s, nb);
  FT_DISPATCH()
#undef X
}

// core gradient partials without the C cache (N = 3, J = R = 16, FP32 only)
static hipError_t core_nc(const ft_plan* P, int m, const ft_params* p, float* partials, hipStream_t s, int* nb) {
  if (P->N != 3 || P->J != 16 || P->R != 16 || bf16(p)) return hipErrorInvalidValue;
  const ModeMeta& M = P->meta[m];
  const ModeDev& D = P->dev[m];
  NoC<3> nc{};
  for (int k = 0; k < 2; ++k) {
    nc.A[k] = p->A[(m + 1 + k) % 3];
    nc.B[k] = p->B[(m + 1 + k) % 3];
  }
  int64_t b = (M.n_segs + 15) / 16;
  b = std::max<int64_t>(1, std::min<int64_t>(b, std::min(kPartials, resident_blocks((const void*)k_core_nc<3>))));
  *nb = (int)b;
  KTimer tm(P, FT_K_SEGSUM, s);
  hipLaunchKernelGGL(k_core_nc<3>, dim3((unsigned)b), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz, D.val, nc,
                     p->A[m], p->B[m], partials);
  return hipGetLastError();
}

hipError_t launch_core_grad(const ft_plan* P, int m, const ft_params* p, const Scratch& S, float* G_out,
                            hipStream_t s) {
  int nb = 0;
  hipError_t e = P->no_c_cache ? core_nc(P, m, p, S.partials, s, &nb)
                               : segsum(P, m, p, S.partials, 0, nullptr, nullptr, s, &nb);
  if (e != hipSuccess) return e;
  return reduce_partials(P, S, nb, nullptr, G_out, 0.f, 0.f, 0.f, 0, s);
}

hipError_t launch_core_update(const ft_plan* P, int m, const ft_params* p, const Scratch& S, double lr, double lam,
                              hipStream_t s) {
  int nb = 0;
  hipError_t e = P->no_c_cache ? core_nc(P, m, p, S.partials, s, &nb)
                               : segsum(P, m, p, S.partials, 0, nullptr, nullptr, s, &nb);
  if (e != hipSuccess) return e;
  const float inv = P->nnz > 0 ? (float)(1.0 / (double)P->nnz) : 0.f;
  return reduce_partials(P, S, nb, p->B[m], nullptr, (float)lr, (float)lam, inv, P->nnz > 0 ? 1 : 0, s);
}

hipError_t launch_loss(const ft_plan* P, const ft_params* p, const Scratch& S, double lam_a, double lam_b,
                       double* out4, hipStream_t s) {
#define X(n, j, r)                                                                             \
  case key(n, j, r):                                                                           \
    return bf16(p) ? loss_impl<n, j, r, uint16_t>(P, p, S.dpartials, lam_a, lam_b, out4, nullptr, s) \
                   : loss_impl<n, j, r, float>(P, p, S.dpartials, lam_a, lam_b, out4, nullptr, s);
  FT_DISPATCH()
#undef X
}

// forward writes no partials (the loss kernel stores xhat only)
hipError_t launch_forward(const ft_plan* P, const ft_params* p, const Scratch&, float* out, hipStream_t s) {
#define X(n, j, r)                                                                             \
  case key(n, j, r):                                                                           \
    return bf16(p) ? loss_impl<n, j, r, uint16_t>(P, p, nullptr, 0.0, 0.0, nullptr, out, s)   \
                   : loss_impl<n, j, r, float>(P, p, nullptr, 0.0, 0.0, nullptr, out, s);
  FT_DISPATCH()
#undef X
}

hipError_t launch_predict(const ft_plan* P, const ft_params* p, const int32_t* coords, int64_t q, float* out,
                          hipStream_t s) {
#define X(n, j, r)                                                                             \
  case key(n, j, r):                                                                           \
    return bf16(p) ? predict_impl<n, r, uint16_t>(p, coords, q, out, s)                       \
                   : predict_impl<n, r, float>(p, coords, q, out, s);
  FT_DISPATCH()
#undef X
}

hipError_t launch_grad(const ft_plan* P, const ft_params* p, const Scratch& S, const float* up, float* const* gA,
                       float* const* gB, hipStream_t s) {
  for (int m = 0; m < P->N; ++m) {
    int nb = 0;
    hipError_t e = segsum(P, m, p, S.partials, up ? 2 : 1, up, S.tseg, s, &nb);
    if (e != hipSuccess) return e;
    switch (P->J * 64 + P->R) {
#define X(n_, j, r)                                                                                        \
  case j * 64 + r:                                                                                         \
    e = bf16(p) ? grad_rows_impl<j, r, uint16_t>(P, m, p, S.tseg, gA[m], s)                               \
                : grad_rows_impl<j, r, float>(P, m, p, S.tseg, gA[m], s);                                 \
    break;
      X(0, 8, 8) X(0, 16, 16) X(0, 32, 32) X(0, 8, 16)
#undef X
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    e = reduce_partials(P, S, nb, nullptr, gB[m], 0.f, 0.f, 0.f, 0, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Scratch of ft_loss_noalloc: the FP64 partials of the loss kernel (at most
// kPartials workgroups) followed by those of the regulariser sums
// (2 N kSumsqBlocks), in a device array that the library holds on every GPU
// it runs on until the process ends.  Host code uses the address looked up
// per device below, never the array's name.
constexpr size_t kNoAllocDoubles = (size_t)kPartials + 2 * FT_MAX_ORDER * kSumsqBlocks;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

size_t noalloc_loss_capacity() { return sizeof(double) * kNoAllocDoubles; }

size_t noalloc_loss_need(const ft_plan* P) {
  return sizeof(double) * ((size_t)kPartials + 2 * (size_t)P->N * kSumsqBlocks);
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device: looked up on the first
// call on each device (with that device current) and kept.
hipError_t noalloc_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* addr = nullptr;
    e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!addr) return hipErrorInvalidSymbol;
    g_noalloc_ptr[dev] = static_cast<double*>(addr);
  }
  *out = g_noalloc_ptr[dev];
  return hipSuccess;
}
}  // namespace

hipError_t launch_loss_noalloc(const ft_plan* P, const ft_params* p, double lam_a, double lam_b, double* out4,
                               hipStream_t s) {
  double* d = nullptr;
  hipError_t e = noalloc_scratch(&d);
  if (e != hipSuccess) return e;
  Scratch S{};
  S.dpartials = d;
  // kernel timing creates events; this path creates nothing
  const UntimedScope untimed;
  return launch_loss(P, p, S, lam_a, lam_b, out4, s);
}

}  // namespace ft
