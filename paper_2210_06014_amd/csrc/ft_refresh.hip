// C refresh (MFMA) and BF16 casts.
#include "ft_device.h"

namespace ft {
namespace {

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

}  // namespace ft
