// HIP kernels of the FasterTucker hot path for CDNA4 (gfx950, wave64).
//
// Lane layouts:
//  * factor pass: a 16-lane DPP row owns one work item; lane l holds element
//    j = l (+16 e) of every J-vector (row of A(m), shared intermediate g, a
//    column of a chunk map) and element r = l (+16 q) of w; values of other
//    lanes are read with DPP row_newbcast, row sums with DPP butterflies;
//  * core, loss, gradient passes: a segment of a row per wavefront, R/4 lanes
//    per element, each lane gathering a 16-byte slice of every C(n) row;
//  * C refresh: v_mfma_f32_16x16x4_f32 tiles of 16 rows.
// No floating-point atomics: every reduction runs in a fixed order.
#include <algorithm>
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "ft_internal.h"

namespace ft {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ int dppi(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
// value of lane L of this lane's 16-lane row (DPP row_newbcast, gfx90a+)
template <int L>
__device__ __forceinline__ float bcast16(float v) {
  return dpp<0x150 + L>(v);
}
template <int L>
__device__ __forceinline__ int bcast16i(int v) {
  return dppi<0x150 + L>(v);
}
// Sum over aligned groups of G lanes (G = 1, 2, 4, 8, 16); every lane of the
// group ends with the same bits (each step adds two equal partial sums).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (G >= 2) v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp<0x141>(v);  // row_half_mirror
  if constexpr (G >= 16) v += dpp<0x140>(v); // row_mirror
  return v;
}


// Fused broadcast-multiply-accumulate: v_fmac_f32_dpp with row_newbcast
// reads src from lane i of the 16-lane row as its first operand, so one
// instruction does what a DPP move plus an FMA would.  The compiler does not
// form these, hence inline assembly.  Each block opens with s_nop 4: five
// wait states cover both DPP hazards of this ISA (a VALU write of the DPP
// source VGPR needs two, a VALU write of EXEC needs five); inside a block no
// instruction writes a register that a later DPP operand of the block reads.
#define FT_BC(n) " row_newbcast:" #n " row_mask:0xf bank_mask:0xf\n\t"
#define FT_DOT(n, op) "v_fmac_f32_dpp %0, %1, %" #op FT_BC(n)
#define FT_AXPY(n, op) "v_fmac_f32_dpp %" #op ", %16, %17" FT_BC(n)
#define FT_AXPY8(n, op) "v_fmac_f32_dpp %" #op ", %8, %9" FT_BC(n)

// acc += sum_{i<16} src[lane i] * v[i]
__device__ __forceinline__ void dot_bcast16(float& acc, float src, const float* v) {
  asm volatile("s_nop 4\n\t" FT_DOT(0, 2) FT_DOT(1, 3) FT_DOT(2, 4) FT_DOT(3, 5) FT_DOT(4, 6) FT_DOT(5, 7)
                   FT_DOT(6, 8) FT_DOT(7, 9) FT_DOT(8, 10) FT_DOT(9, 11) FT_DOT(10, 12) FT_DOT(11, 13)
                       FT_DOT(12, 14) FT_DOT(13, 15) FT_DOT(14, 16) FT_DOT(15, 17)
               : "+v"(acc)
               : "v"(src), "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]),
                 "v"(v[8]), "v"(v[9]), "v"(v[10]), "v"(v[11]), "v"(v[12]), "v"(v[13]), "v"(v[14]), "v"(v[15]));
}
// acc += sum_{i<8} src[lane i] * v[i]
__device__ __forceinline__ void dot_bcast8(float& acc, float src, const float* v) {
  asm volatile("s_nop 4\n\t" FT_DOT(0, 2) FT_DOT(1, 3) FT_DOT(2, 4) FT_DOT(3, 5) FT_DOT(4, 6) FT_DOT(5, 7)
                   FT_DOT(6, 8) FT_DOT(7, 9)
               : "+v"(acc)
               : "v"(src), "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]));
}
// v[i] += src[lane i] * t, i < 16
__device__ __forceinline__ void axpy_bcast16(float* v, float src, float t) {
  asm volatile("s_nop 4\n\t" FT_AXPY(0, 0) FT_AXPY(1, 1) FT_AXPY(2, 2) FT_AXPY(3, 3) FT_AXPY(4, 4) FT_AXPY(5, 5)
                   FT_AXPY(6, 6) FT_AXPY(7, 7) FT_AXPY(8, 8) FT_AXPY(9, 9) FT_AXPY(10, 10) FT_AXPY(11, 11)
                       FT_AXPY(12, 12) FT_AXPY(13, 13) FT_AXPY(14, 14) FT_AXPY(15, 15)
               : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7]),
                 "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]), "+v"(v[14]), "+v"(v[15])
               : "v"(src), "v"(t));
}
// v[i] += src[lane i] * t, i < 8
__device__ __forceinline__ void axpy_bcast8(float* v, float src, float t) {
  asm volatile("s_nop 4\n\t" FT_AXPY8(0, 0) FT_AXPY8(1, 1) FT_AXPY8(2, 2) FT_AXPY8(3, 3) FT_AXPY8(4, 4)
                   FT_AXPY8(5, 5) FT_AXPY8(6, 6) FT_AXPY8(7, 7)
               : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7])
               : "v"(src), "v"(t));
}
template <int K>
__device__ __forceinline__ void dot_bcast(float& acc, float src, const float* v) {
  static_assert(K == 8 || K == 16, "row broadcasts cover 8 or 16 lanes");
  if constexpr (K == 16) dot_bcast16(acc, src, v); else dot_bcast8(acc, src, v);
}
template <int K>
__device__ __forceinline__ void axpy_bcast(float* v, float src, float t) {
  static_assert(K == 8 || K == 16, "row broadcasts cover 8 or 16 lanes");
  if constexpr (K == 16) axpy_bcast16(v, src, t); else axpy_bcast8(v, src, t);
}

// Parameter storage: float (FP32) or uint16_t holding BF16 bits.  BF16 is
// widened exactly by a 16-bit shift; all arithmetic is FP32.
__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(uint16_t x) { return __uint_as_float((uint32_t)x << 16); }

template <int N, class T = float>
struct CPtrs {
  const T* p[N > 1 ? N - 1 : 1];
};

// four consecutive values starting at p (16-byte aligned for float, 8-byte for BF16)
__device__ __forceinline__ floatx4 load4(const float* p) { return *reinterpret_cast<const floatx4*>(p); }
__device__ __forceinline__ floatx4 load4(const uint16_t* p) {
  const uint2 u = *reinterpret_cast<const uint2*>(p);
  floatx4 r;
  r[0] = __uint_as_float(u.x << 16);
  r[1] = __uint_as_float(u.x & 0xFFFF0000u);
  r[2] = __uint_as_float(u.y << 16);
  r[3] = __uint_as_float(u.y & 0xFFFF0000u);
  return r;
}

// ---------------------------------------------------------------------------
// C = A B  (I x J) (J x R), FP32 MFMA 16x16x4.  One wavefront per 16 rows.
// Operand layout of v_mfma_f32_16x16x4_f32: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register v of lane l is D[4*(l/16)+v][l%16].
template <int J, int R>
__global__ __launch_bounds__(256) void k_refresh(const float* __restrict__ A, const float* __restrict__ B,
                                                 float* __restrict__ C, int64_t I) {
  const int lane = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (row0 >= I) return;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t ia = row0 + li;
  constexpr int CT = (R + 15) / 16;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    const int col = ct * 16 + li;
#pragma unroll
    for (int kb = 0; kb < J / 4; ++kb) {
      const int k = kb * 4 + lk;
      const float a = ia < I ? A[ia * J + k] : 0.f;
      const float b = col < R ? B[k * R + col] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = row0 + lk * 4 + v;
      if (r < I && col < R) C[r * R + col] = acc[v];
    }
  }
}

// BF16 storage: C16 = bf16(A16 B16) with v_mfma_f32_16x16x16_bf16 (FP32
// accumulation).  Lane l supplies A[l%16][4(l/16) .. 4(l/16)+3] and
// B[4(l/16) .. +3][l%16]; the result layout is that of the FP32 tile.
typedef short shortx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even on the upper 16 bits (IEEE-754 binary32 -> bfloat16); NaN stays NaN
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <int J, int R>
__global__ __launch_bounds__(256) void k_refresh_bf16(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B,
                                                      uint16_t* __restrict__ C, int64_t I) {
  const int lane = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (row0 >= I) return;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t ia = row0 + li;
  constexpr int CT = (R + 15) / 16;
  constexpr int KB = (J + 15) / 16;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    const int col = ct * 16 + li;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      shortx4 a, b;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = kb * 16 + lk * 4 + u;
        a[u] = (ia < I && k < J) ? (short)A[ia * J + k] : (short)0;
        b[u] = (col < R && k < J) ? (short)B[k * R + col] : (short)0;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = row0 + lk * 4 + v;
      if (r < I && col < R) C[r * R + col] = f2bf(acc[v]);
    }
  }
}

__global__ __launch_bounds__(256) void k_cast_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                                   int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
    dst[k] = f2bf(src[k]);
}

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

// value at byte offset `off` of a C table (uniform base + 32-bit offset: the
// scalar-base addressing form; every table is far below 4 GB)
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

// The same w without the C cache (FastTucker's cost, kept for the Table 5
// comparison): each C(n) row is formed on use as A(n)[i, :] B(n).  Lane j
// loads A(n)[i, j]; a row broadcast against the lane's column of B(n) then
// gives C(n)[i, r] in lane r (J = R = 16).
template <int N>
struct NoC {
  const float* A[N > 1 ? N - 1 : 1];  // A(n) of the other modes, in table order
  const float* B[N > 1 ? N - 1 : 1];
};

template <int N>
__device__ __forceinline__ void load_nc_cols(const NoC<N>& nc, int l, float (&Bc)[N > 1 ? N - 1 : 1][16]) {
#pragma unroll
  for (int k = 0; k < N - 1; ++k)
#pragma unroll
    for (int j = 0; j < 16; ++j) Bc[k][j] = nc.B[k][j * 16 + l];
}

// ix[k]: row index of element (lane t)'s k-th other mode
template <int N>
__device__ __forceinline__ void gather_w_nc(const NoC<N>& nc, const float (&Bc)[N > 1 ? N - 1 : 1][16],
                                            const int (&ix)[N > 1 ? N - 1 : 1], int l, int t0, int len,
                                            float (&w)[16][1]) {
  float av[16][N - 1];
  static_for<0, 16>([&](auto S) {
    constexpr int s = decltype(S)::value;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) av[s][k] = nc.A[k][(int64_t)bcast16i<s>(ix[k]) * 16 + l];
  });
  static_for<0, 16>([&](auto S) {
    constexpr int s = decltype(S)::value;
    float prod = 0.f;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
      float c = 0.f;
      dot_bcast16(c, av[s][k], Bc[k]);
      prod = k == 0 ? c : prod * c;
    }
    w[s][0] = (t0 + s) < len ? prod : 0.f;
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
      ixb[b][k] = len[b] > 0 ? fib_idx[(int64_t)k * nfib + f] * (int)(R * sizeof(T)) : 0;
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

template <int N, int J, int R, class T, bool FIB, bool NC = false>
__global__ __launch_bounds__(256) void k_factor_apply(const FItem* __restrict__ items, int64_t n_items,
                                                      const int32_t* __restrict__ idx, int64_t nnz,
                                                      const float* __restrict__ val, CPtrs<N, T> cp,
                                                      const T* __restrict__ Bm, float* __restrict__ Am,
                                                      float* __restrict__ hvec, float lr, float c1,
                                                      const int32_t* __restrict__ fid, const float* __restrict__ gfib,
                                                      NoC<N> nc) {
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
  // One item per 16-lane group: the four groups of a wavefront take four
  // consecutive items (similar lengths, the lists are sorted).
  const int64_t gid = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
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
        ix[k] = it.len > 0 ? idx[(int64_t)k * nnz + p] * (NC ? 1 : (int)(R * sizeof(T))) : 0;
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
  if (it.len > 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = l + 16 * e;
      if (j < J) {
        if (it.kind == ITEM_LIGHT)
          Am[(int64_t)it.row * J + j] = (float)a[e];
        else
          hvec[(int64_t)it.slot * J + j] = (float)a[e];
      }
    }
  }
}

// Chunk maps.  With rho = 1 - lr lam and gp = lr / rho, one step is
//     a <- rho (I - gp g g^T) a + lr x g.
// A chunk of T steps is the affine map a -> rho^T (I + Nm) a + v with
//     Nm <- Nm - gp g (g + Nm^T g)^T     (Nm = prod (I - gp g g^T) - I)
//     v  <- v + (-lr lam) v + lr (x - v.g) g
// (v is the state reached from a = 0).  Lane j keeps column j of Nm.
template <int N, int J, int R, class T, bool FIB, bool NC = false>
__global__ __launch_bounds__(256) void k_factor_compose(const FItem* __restrict__ items, int64_t n_items,
                                                        const int32_t* __restrict__ idx, int64_t nnz,
                                                        const float* __restrict__ val, CPtrs<N, T> cp,
                                                        const T* __restrict__ Bm, float* __restrict__ maps,
                                                        double* __restrict__ map_scale, float lr, float c1, float gp,
                                                        double rho, const int32_t* __restrict__ fid,
                                                        const float* __restrict__ gfib, NoC<N> nc) {
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
  // One item per 16-lane group: the four groups of a wavefront take four
  // consecutive items (similar lengths, the lists are sorted).
  const int64_t gid = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
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
        ix[k] = it.len > 0 ? idx[(int64_t)k * nnz + p] * (NC ? 1 : (int)(R * sizeof(T))) : 0;
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
  constexpr int RMAX = (F / 2 * J * J + 255) / 256;  // matrix entries per thread at the widest level
  constexpr int VMAX = (F / 2 * J + 255) / 256;      // vector entries per thread at the widest level
  __shared__ float buf[F * MS];
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
    float res[RMAX];
#pragma unroll
    for (int u = 0; u < RMAX; ++u) {
      const int e = t + 256 * u;
      if (e < pairs * J * J) {
        const int pr = e / (J * J), ij = e % (J * J);
        const int i = ij % J, j = ij / J;
        const float* Na = buf + (2 * pr * stride) * MS;
        const float* Nb = Na + stride * MS;
        float acc = 0.f;
#pragma unroll
        for (int q = 0; q < J; ++q) acc = fmaf(Nb[q * J + i], Na[j * J + q], acc);
        res[u] = (Na[ij] + Nb[ij]) + acc;
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
    for (int u = 0; u < RMAX; ++u) {
      const int e = t + 256 * u;
      if (e < pairs * J * J) {
        const int pr = e / (J * J), ij = e % (J * J);
        buf[(2 * pr * stride) * MS + ij] = res[u];
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

// ---------------------------------------------------------------------------
// dispatch

#define FT_CONFIGS(X)                                                                                       \
  X(3, 8, 8) X(3, 16, 16) X(3, 32, 32) X(4, 8, 8) X(4, 32, 32) X(8, 8, 16) X(5, 32, 32) X(6, 32, 32) X(7, 32, 32) \
      X(8, 32, 32) X(9, 32, 32) X(10, 32, 32)

constexpr int key(int N, int J, int R) { return (N * 64 + J) * 64 + R; }

// Typed views of the parameter set: FP32 storage reads A, B, C; BF16 storage
// reads the BF16 copies A16, B16, C16 (the FP32 masters A, B take the updates).
template <class T>
struct Store;
template <>
struct Store<float> {
  static const float* A(const ft_params* p, int n) { return p->A[n]; }
  static const float* B(const ft_params* p, int n) { return p->B[n]; }
  static const float* C(const ft_params* p, int n) { return p->C[n]; }
};
template <>
struct Store<uint16_t> {
  static const uint16_t* A(const ft_params* p, int n) { return (const uint16_t*)p->A16[n]; }
  static const uint16_t* B(const ft_params* p, int n) { return (const uint16_t*)p->B16[n]; }
  static const uint16_t* C(const ft_params* p, int n) { return (const uint16_t*)p->C16[n]; }
};

template <int N, class T>
CPtrs<N, T> others(const ft_params* p, int m) {
  CPtrs<N, T> c{};
  for (int k = 0; k < N - 1; ++k) c.p[k] = Store<T>::C(p, (m + 1 + k) % N);
  return c;
}

// Workgroups that fit on the device at once for a 256-thread kernel (from the
// occupancy query, cached per kernel).  The segment passes, whose wavefronts
// each walk a fixed set of segments, launch at most this many.
int resident_blocks(const void* kernel) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto f = cache.find(kernel);
  if (f != cache.end()) return f->second;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || cus <= 0 || per_cu <= 0) {
    cus = 256;
    per_cu = 2;
  }
  const int r = cus * per_cu;
  cache.emplace(kernel, r);
  return r;
}

// One item per 16-lane group: the hardware dispatcher balances the items
// (measured faster than a grid-stride loop, which also costs registers).
unsigned factor_blocks(const void* kernel, int64_t n_items) {
  (void)kernel;
  return (unsigned)std::max<int64_t>(1, (n_items + 15) / 16);
}

template <int N, int J, int R, class T, bool FIB, bool NC = false>
hipError_t factor_launch(const ft_plan* P, int m, const ft_params* p, double lr, double lam, hipStream_t s) {
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
                       0, s, D.fib_idx, M.n_fibers, cp, Bm, P->gfib);
  }
  if (M.n_compose > 0) {
    KTimer tm(P, FT_K_FACTOR_COMPOSE, s);
    hipLaunchKernelGGL((k_factor_compose<N, J, R, T, FIB, NC>),
                       dim3(factor_blocks((const void*)k_factor_compose<N, J, R, T, FIB, NC>, M.n_compose)), dim3(256),
                       0, s, D.compose, M.n_compose, D.idx, P->nnz, D.val, cp, Bm, P->maps, P->map_scale, flr, c1, gp,
                       rho, D.fid, P->gfib, nc);
  }
  if (M.n_apply > 0) {
    KTimer tm(P, FT_K_FACTOR_APPLY, s);
    hipLaunchKernelGGL((k_factor_apply<N, J, R, T, FIB, NC>),
                       dim3(factor_blocks((const void*)k_factor_apply<N, J, R, T, FIB, NC>, M.n_apply)), dim3(256), 0,
                       s, D.apply, M.n_apply, D.idx, P->nnz, D.val, cp, Bm, p->A[m], P->hvec, flr, c1, D.fid, P->gfib,
                       nc);
  }
  for (size_t L = 0; L < M.level_len.size(); ++L) {
    KTimer tm(P, FT_K_COMBINE, s);
    const int64_t nc = M.level_ncomp[L], nf = M.level_len[L] - nc;
    if (nc > 0)
      hipLaunchKernelGGL((k_combine<J>), dim3((unsigned)nc), dim3(256), 0, s, D.levels + M.level_off[L], P->maps,
                         P->map_scale);
    if (nf > 0)
      hipLaunchKernelGGL((k_combine_final<J>), dim3((unsigned)((nf + 15) / 16)), dim3(256), 0, s,
                         D.levels + M.level_off[L] + nc, nf, P->maps, P->map_scale, P->hvec, p->A[m]);
  }
  return hipGetLastError();
}

template <int N, int J, int R, class T>
hipError_t factor_impl(const ft_plan* P, int m, const ft_params* p, double lr, double lam, hipStream_t s) {
  if (P->no_c_cache) {
    if constexpr (N == 3 && J == 16 && R == 16 && std::is_same<T, float>::value)
      return factor_launch<N, J, R, T, false, true>(P, m, p, lr, lam, s);
    else
      return hipErrorInvalidValue;  // rejected at plan creation and in the parameter checks
  }
  return P->meta[m].use_fiber ? factor_launch<N, J, R, T, true>(P, m, p, lr, lam, s)
                              : factor_launch<N, J, R, T, false>(P, m, p, lr, lam, s);
}

hipError_t reduce_partials(const ft_plan* P, int nparts, float* Bm, float* Gout, float lr, float lam, float inv,
                           int update, hipStream_t s) {
  KTimer tm(P, FT_K_REDUCE, s);
  const int JR = P->J * P->R;
  const int nfold = (nparts + kFold - 1) / kFold;
  float* folded = P->partials + (int64_t)kPartials * JR;
  if (nfold > 0) hipLaunchKernelGGL(k_fold_partials, dim3(nfold), dim3(256), 0, s, P->partials, nparts, JR, folded);
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
hipError_t segsum_impl(const ft_plan* P, int m, const ft_params* p, int mode, const float* up, float* tseg,
                       hipStream_t s, int* nblocks) {
  const ModeMeta& M = P->meta[m];
  const ModeDev& D = P->dev[m];
  const CPtrs<N, T> cp = others<N, T>(p, m);
  const T* Cm = Store<T>::C(p, m);
  const T* Am = Store<T>::A(p, m);
  const void* kern = mode == 0 ? (const void*)k_segsum<N, J, R, 0, T>
                     : mode == 1 ? (const void*)k_segsum<N, J, R, 1, T> : (const void*)k_segsum<N, J, R, 2, T>;
  const int nb = seg_blocks(kern, M.n_segs);
  *nblocks = nb;
  KTimer tm(P, FT_K_SEGSUM, s);
  if (mode == 0)
    hipLaunchKernelGGL((k_segsum<N, J, R, 0, T>), dim3(nb), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz, D.val,
                       cp, Cm, Am, nullptr, nullptr, P->partials, tseg);
  else if (mode == 1)
    hipLaunchKernelGGL((k_segsum<N, J, R, 1, T>), dim3(nb), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz, D.val,
                       cp, Cm, Am, nullptr, nullptr, P->partials, tseg);
  else
    hipLaunchKernelGGL((k_segsum<N, J, R, 2, T>), dim3(nb), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz, D.val,
                       cp, Cm, Am, up, D.perm, P->partials, tseg);
  return hipGetLastError();
}

template <int N, int J, int R, class T>
hipError_t loss_impl(const ft_plan* P, const ft_params* p, double lam_a, double lam_b, double* out4, float* xout,
                     hipStream_t s) {
  const ModeMeta& M = P->meta[0];
  const ModeDev& D = P->dev[0];
  const CPtrs<N, T> cp = others<N, T>(p, 0);
  const int nb = seg_blocks((const void*)k_loss<N, R, T>, M.n_segs);
  {
    KTimer tm(P, FT_K_LOSS, s);
    hipLaunchKernelGGL((k_loss<N, R, T>), dim3(nb), dim3(256), 0, s, D.segs, M.n_segs, D.idx, P->nnz, D.val, cp,
                       Store<T>::C(p, 0), out4 ? P->dpartials : nullptr, D.perm, xout);
  }
  if (!out4) return hipGetLastError();
  // the regularisers of Eq. (6) are taken on the FP32 masters
  KTimer tm(P, FT_K_REDUCE, s);
  double* rpart = P->dpartials + kPartials;
  for (int n = 0; n < N; ++n)
    hipLaunchKernelGGL(k_sumsq, dim3(kSumsqBlocks), dim3(256), 0, s, p->A[n], P->desc.dims[n] * J,
                       rpart + n * kSumsqBlocks);
  for (int n = 0; n < N; ++n)
    hipLaunchKernelGGL(k_sumsq, dim3(kSumsqBlocks), dim3(256), 0, s, p->B[n], (int64_t)J * R,
                       rpart + (N + n) * kSumsqBlocks);
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, P->dpartials, nb, rpart, N * kSumsqBlocks,
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
hipError_t grad_rows_impl(const ft_plan* P, int m, const ft_params* p, float* gA, hipStream_t s) {
  const int64_t I = P->desc.dims[m];
  const unsigned gb = (unsigned)((I * J + 255) / 256);
  if (gb > 0)
    hipLaunchKernelGGL((k_grad_rows<J, R, T>), dim3(gb), dim3(256), 0, s, P->dev[m].seg_ptr, P->tseg,
                       Store<T>::B(p, m), gA, I);
  return hipGetLastError();
}

bool bf16(const ft_params* p) { return p->storage == FT_STORE_BF16; }

}  // namespace

int max_fanin(int J) { return J <= 8 ? combine_fanin<8>() : J <= 16 ? combine_fanin<16>() : combine_fanin<32>(); }

bool supported(int N, int J, int R) {
  switch (key(N, J, R)) {
#define X(n, j, r) \
  case key(n, j, r): return true;
    FT_CONFIGS(X)
#undef X
    default: return false;
  }
}

hipError_t launch_refresh(const ft_plan* P, int n, const ft_params* p, hipStream_t s) {
  const int64_t I = P->desc.dims[n];
  const unsigned nb = (unsigned)(((I + 15) / 16 + 3) / 4);
  KTimer tm(P, FT_K_REFRESH, s);
  if (bf16(p)) {
    // BF16 copies of the masters (round to nearest even), then C16 = bf16(A16 B16)
    const int64_t na = I * P->J, nbm = (int64_t)P->J * P->R;
    hipLaunchKernelGGL(k_cast_bf16, dim3((unsigned)std::min<int64_t>((na + 255) / 256, 4096) + (na == 0)), dim3(256),
                       0, s, p->A[n], (uint16_t*)p->A16[n], na);
    hipLaunchKernelGGL(k_cast_bf16, dim3((unsigned)((nbm + 255) / 256)), dim3(256), 0, s, p->B[n],
                       (uint16_t*)p->B16[n], nbm);
    if (nb == 0) return hipGetLastError();
    switch (P->J * 64 + P->R) {
#define X(n_, j, r)                                                                                       \
  case j * 64 + r:                                                                                        \
    hipLaunchKernelGGL((k_refresh_bf16<j, r>), dim3(nb), dim3(256), 0, s, (const uint16_t*)p->A16[n],    \
                       (const uint16_t*)p->B16[n], (uint16_t*)p->C16[n], I);                              \
    return hipGetLastError();
      X(0, 8, 8) X(0, 16, 16) X(0, 32, 32) X(0, 8, 16)
#undef X
      default: return hipErrorInvalidValue;
    }
  }
  if (nb == 0) return hipSuccess;
  switch (P->J * 64 + P->R) {
#define X(n_, j, r)                                                                                           \
  case j * 64 + r:                                                                                            \
    hipLaunchKernelGGL((k_refresh<j, r>), dim3(nb), dim3(256), 0, s, p->A[n], p->B[n], p->C[n], I);          \
    return hipGetLastError();
    X(0, 8, 8) X(0, 16, 16) X(0, 32, 32) X(0, 8, 16)
#undef X
    default: return hipErrorInvalidValue;
  }
}

#define FT_DISPATCH(CALL)                                            \
  switch (key(P->N, P->J, P->R)) {                                   \
    FT_CONFIGS(X)                                                    \
    default: return hipErrorInvalidValue;                            \
  }

hipError_t launch_factor(const ft_plan* P, int m, const ft_params* p, double lr, double lam, hipStream_t s) {
#define X(n, j, r)                                                                             \
  case key(n, j, r):                                                                           \
    return bf16(p) ? factor_impl<n, j, r, uint16_t>(P, m, p, lr, lam, s)                      \
                   : factor_impl<n, j, r, float>(P, m, p, lr, lam, s);
  FT_DISPATCH()
#undef X
}

static hipError_t segsum(const ft_plan* P, int m, const ft_params* p, int mode, const float* up, float* tseg,
                         hipStream_t s, int* nb) {
#define X(n, j, r)                                                                             \
  case key(n, j, r):                                                                           \
    return bf16(p) ? segsum_impl<n, j, r, uint16_t>(P, m, p, mode, up, tseg, s, nb)           \
                   : segsum_impl<n, j, r, float>(P, m, p, mode, up, tseg, s, nb);
  FT_DISPATCH()
#undef X
}

// core gradient partials without the C cache (N = 3, J = R = 16, FP32 only)
static hipError_t core_nc(const ft_plan* P, int m, const ft_params* p, hipStream_t s, int* nb) {
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
                     p->A[m], p->B[m], P->partials);
  return hipGetLastError();
}

hipError_t launch_core_grad(const ft_plan* P, int m, const ft_params* p, hipStream_t s) {
  int nb = 0;
  hipError_t e = P->no_c_cache ? core_nc(P, m, p, s, &nb) : segsum(P, m, p, 0, nullptr, nullptr, s, &nb);
  if (e != hipSuccess) return e;
  return reduce_partials(P, nb, nullptr, P->gbuf, 0.f, 0.f, 0.f, 0, s);
}

hipError_t launch_core_update(const ft_plan* P, int m, const ft_params* p, double lr, double lam, float* G_out,
                              hipStream_t s) {
  int nb = 0;
  hipError_t e = P->no_c_cache ? core_nc(P, m, p, s, &nb) : segsum(P, m, p, 0, nullptr, nullptr, s, &nb);
  if (e != hipSuccess) return e;
  const float inv = P->nnz > 0 ? (float)(1.0 / (double)P->nnz) : 0.f;
  return reduce_partials(P, nb, p->B[m], G_out, (float)lr, (float)lam, inv, P->nnz > 0 ? 1 : 0, s);
}

hipError_t launch_loss(const ft_plan* P, const ft_params* p, double lam_a, double lam_b, double* out4, hipStream_t s) {
#define X(n, j, r)                                                                             \
  case key(n, j, r):                                                                           \
    return bf16(p) ? loss_impl<n, j, r, uint16_t>(P, p, lam_a, lam_b, out4, nullptr, s)       \
                   : loss_impl<n, j, r, float>(P, p, lam_a, lam_b, out4, nullptr, s);
  FT_DISPATCH()
#undef X
}

hipError_t launch_forward(const ft_plan* P, const ft_params* p, float* out, hipStream_t s) {
#define X(n, j, r)                                                                             \
  case key(n, j, r):                                                                           \
    return bf16(p) ? loss_impl<n, j, r, uint16_t>(P, p, 0.0, 0.0, nullptr, out, s)            \
                   : loss_impl<n, j, r, float>(P, p, 0.0, 0.0, nullptr, out, s);
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

hipError_t launch_grad(const ft_plan* P, const ft_params* p, const float* up, float* const* gA, float* const* gB,
                       hipStream_t s) {
  for (int m = 0; m < P->N; ++m) {
    int nb = 0;
    hipError_t e = segsum(P, m, p, up ? 2 : 1, up, P->tseg, s, &nb);
    if (e != hipSuccess) return e;
    switch (P->J * 64 + P->R) {
#define X(n_, j, r)                                                                                        \
  case j * 64 + r:                                                                                         \
    e = bf16(p) ? grad_rows_impl<j, r, uint16_t>(P, m, p, gA[m], s) : grad_rows_impl<j, r, float>(P, m, p, gA[m], s); \
    break;
      X(0, 8, 8) X(0, 16, 16) X(0, 32, 32) X(0, 8, 16)
#undef X
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    e = reduce_partials(P, nb, nullptr, gB[m], 0.f, 0.f, 0.f, 0, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ft
