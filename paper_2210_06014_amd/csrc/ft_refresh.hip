// C refresh (MFMA) and BF16 casts.
#include "ft_device.h"

namespace ft {
namespace {

// ---------------------------------------------------------------------------
// C = A B  (I x J) (J x R) on the matrix cores, TPW tiles of 16 rows per
// wavefront.  The refresh streams A in and C out (a few flops per byte), so
// the layout is chosen for the loads: the sum over k may run in any order,
// and lane (i, g) of a tile (row i = lane % 16, group g = lane / 16) takes
// the k values whose A entries are contiguous in its row, so that A arrives
// in 16-byte loads covering whole row pieces; every load of a wavefront is
// issued before its first MFMA.

constexpr int kRefreshTiles = 4;  // 16-row tiles per wavefront

// FP32, v_mfma_f32_16x16x4_f32: lane (i, g) supplies A[i][k] and B[k][col]
// for one k per instruction and receives D[4 g + v][col], col = lane % 16.
// For J a multiple of 16 its k values are 16 h + 4 g + u (h < J / 16,
// u < 4: float4 loads); for J = 8 they are 2 g + u.
template <int J>
__device__ __forceinline__ int refresh_k(int g, int kb) {
  if constexpr (J % 16 == 0)
    return 16 * (kb / 4) + 4 * g + (kb % 4);
  else
    return (J / 4) * g + kb;
}

template <int J, int R>
__global__ __launch_bounds__(256) void k_refresh(const float* __restrict__ A, const float* __restrict__ B,
                                                 float* __restrict__ C, int64_t I) {
  static_assert(J % 4 == 0, "J is a multiple of 4");
  constexpr int KPL = J / 4;  // k values per lane
  constexpr int CT = (R + 15) / 16;
  constexpr int TPW = kRefreshTiles;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int64_t tile0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TPW;
  if (tile0 * 16 >= I) return;
  float b[CT][KPL];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = ct * 16 + li;
#pragma unroll
    for (int kb = 0; kb < KPL; ++kb) b[ct][kb] = col < R ? B[refresh_k<J>(lg, kb) * R + col] : 0.f;
  }
  float a[TPW][KPL];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int64_t row = (tile0 + t) * 16 + li;
    const bool ok = row < I;
    const float* ar = A + (ok ? row : 0) * J;
    if constexpr (J % 16 == 0) {
#pragma unroll
      for (int h = 0; h < J / 16; ++h) {
        const floatx4 v = *reinterpret_cast<const floatx4*>(ar + 16 * h + 4 * lg);
#pragma unroll
        for (int u = 0; u < 4; ++u) a[t][4 * h + u] = ok ? v[u] : 0.f;
      }
    } else {
#pragma unroll
      for (int kb = 0; kb < KPL; ++kb) a[t][kb] = ok ? ar[refresh_k<J>(lg, kb)] : 0.f;
    }
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int64_t row0 = (tile0 + t) * 16;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < KPL; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][kb], b[ct][kb], acc, 0, 0, 0);
      const int col = ct * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + lg * 4 + v;
        if (r < I && col < R) C[r * R + col] = acc[v];
      }
    }
  }
}

// BF16 storage: C16 = bf16(A16 B16) with v_mfma_f32_16x16x16_bf16 (FP32
// accumulation).  Lane (i, g) supplies four k values per instruction: with
// J a multiple of 32 they are 8 g + 4 kb + u (one 16-byte load of 8 BF16
// values per row covers both instructions), otherwise 16 kb + 4 g + u; k
// beyond J supplies zeros.  The result layout is that of the FP32 tile.
typedef short shortx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even on the upper 16 bits (IEEE-754 binary32 -> bfloat16); NaN stays NaN
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <int J>
__device__ __forceinline__ int refresh_k16(int g, int kb, int u) {
  if constexpr (J % 32 == 0)
    return 32 * (kb / 2) + 8 * g + 4 * (kb % 2) + u;
  else
    return 16 * kb + 4 * g + u;
}

template <int J, int R>
__global__ __launch_bounds__(256) void k_refresh_bf16(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B,
                                                      uint16_t* __restrict__ C, int64_t I) {
  constexpr int CT = (R + 15) / 16;
  constexpr int KB = (J + 15) / 16;
  constexpr int TPW = kRefreshTiles;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int64_t tile0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TPW;
  if (tile0 * 16 >= I) return;
  shortx4 b[CT][KB];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int col = ct * 16 + li;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = refresh_k16<J>(lg, kb, u);
        b[ct][kb][u] = (col < R && k < J) ? (short)B[k * R + col] : (short)0;
      }
  }
  shortx4 a[TPW][KB];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int64_t row = (tile0 + t) * 16 + li;
    const bool ok = row < I;
    const uint16_t* ar = A + (ok ? row : 0) * J;
    if constexpr (J % 32 == 0) {
#pragma unroll
      for (int h = 0; h < J / 32; ++h) {
        const uint4 v = *reinterpret_cast<const uint4*>(ar + 32 * h + 8 * lg);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a[t][2 * h + q / 2][2 * (q % 2)] = ok ? (short)(w[q] & 0xFFFFu) : (short)0;
          a[t][2 * h + q / 2][2 * (q % 2) + 1] = ok ? (short)(w[q] >> 16) : (short)0;
        }
      }
    } else {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = refresh_k16<J>(lg, kb, u);
          a[t][kb][u] = (ok && k < J) ? (short)ar[k] : (short)0;
        }
    }
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int64_t row0 = (tile0 + t) * 16;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[t][kb], b[ct][kb], acc, 0, 0, 0);
      const int col = ct * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + lg * 4 + v;
        if (r < I && col < R) C[r * R + col] = f2bf(acc[v]);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_cast_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                                   int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
    dst[k] = f2bf(src[k]);
}

}  // namespace

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
  const int64_t waves = ((I + 15) / 16 + kRefreshTiles - 1) / kRefreshTiles;
  const unsigned nb = (unsigned)((waves + 3) / 4);
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

}  // namespace ft
