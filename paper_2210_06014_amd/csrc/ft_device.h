// Device helpers and host-side dispatch pieces shared by the kernel files
// (ft_refresh.hip, ft_factor.hip, ft_segment.hip).
//
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
#pragma once
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

bool bf16(const ft_params* p) { return p->storage == FT_STORE_BF16; }

#define FT_DISPATCH(CALL)                                            \
  switch (key(P->N, P->J, P->R)) {                                   \
    FT_CONFIGS(X)                                                    \
    default: return hipErrorInvalidValue;                            \
  }

}  // namespace
}  // namespace ft
