// hot_probes.hip -- micro-benchmarks of the pipes that bound the direct-sum passes.
//
// The direct passes of the solver (Eq. 1 and Eq. 3 with Delta from Eq. 2 recomputed per
// (pixel, trap) pair) are bound by FP32 vector issue: per term two FMAs form the phase, the
// hardware sin and cos turn it into a phasor, and two FMAs accumulate it.  The roofline the
// benchmark quotes rests on three measured facts about gfx950, which these kernels measure on
// the machine they run on:
//   * the FP32 FMA issue rate (one wave64 instruction per SIMD per 4 shader cycles at peak);
//   * the V_SIN_F32 / V_COS_F32 issue rate;
//   * whether the two overlap: a stream with the term's exact mix (4 FMA : 1 sin : 1 cos) runs
//     at the sum of the two costs (no overlap) or faster;
// The separable variant runs both passes as FP32 matrix products (V_MFMA_F32_16X16X4_F32), so
// the matrix pipe's issue rate is measured too: with four independent accumulators per wave,
// with one accumulator (each product waits for the previous one's result), and for the 32x32x2
// shape;
// each at 1, 2, 4 and 8 waves per SIMD, together with the shader clock the waves ran at
// (s_memtime counts shader cycles, s_memrealtime a constant 100 MHz clock).  Every wave writes
// its own clock stamps (vector stores) and one value derived from all its results, so no work
// can be removed by the compiler.
#include "hot_internal.h"

namespace hot {

namespace {

constexpr int kProbeUnroll = 16;

__device__ __forceinline__ unsigned long long shader_clock() { return __builtin_amdgcn_s_memtime(); }
__device__ __forceinline__ unsigned long long real_clock() { return __builtin_amdgcn_s_memrealtime(); }

// KIND 0: FMA only, 8 independent chains (128 FMAs per repetition).
// KIND 1: sin / cos only, 8 independent chains (128 transcendentals per repetition).
// KIND 2: the term of a direct pass, 16 per repetition: t = fma(g, U^2, fma(a, U, c));
//         re += w cos t; im += w sin t (64 FMAs + 32 transcendentals per repetition, plus one
//         add that moves c on).
// KIND 3: V_MFMA_F32_16X16X4_F32, 4 independent accumulators (16 products per repetition).
// KIND 4: V_MFMA_F32_16X16X4_F32, one accumulator: every product depends on the one before (16 per
//         repetition).
// KIND 5: V_MFMA_F32_32X32X2_F32, 4 independent accumulators (16 products per repetition).
// KIND 6: KIND 3's 16 products with 64 independent sin/cos beside them per repetition (512 matrix
//         cycles against 512 transcendental cycles per SIMD if each wave ran alone): whether the
//         transcendental pipe runs while the matrix pipe works.
typedef float probe_f32x4 __attribute__((ext_vector_type(4)));
typedef float probe_f32x16 __attribute__((ext_vector_type(16)));

template <int KIND>
__global__ void __launch_bounds__(1024)
k_probe(long long reps, float seed, float* __restrict__ sink, unsigned long long* __restrict__ stamps) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const unsigned long long c0 = shader_clock(), r0 = real_clock();
  float out = 0.0f;
  if constexpr (KIND == 0) {
    // a[i] += m x[i]: the accumulate form (v_fmac_f32, register operands only)
    float a[8], x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      a[i] = seed + 0.001f * (float)(lane + i);
      x[i] = 0.5f * seed + 0.002f * (float)i;
    }
    const float m = 1.0e-7f * seed;
    for (long long r = 0; r < reps; ++r) {
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = __builtin_fmaf(m, x[i], a[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) out += a[i];
  } else if constexpr (KIND == 1) {
    float s[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = seed * 0.01f + 0.003f * (float)(lane + i);
    for (long long r = 0; r < reps; ++r) {
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u) {
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] = (i & 1) ? __builtin_amdgcn_cosf(s[i]) : __builtin_amdgcn_sinf(s[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) out += s[i];
  } else if constexpr (KIND == 6) {
    probe_f32x4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = probe_f32x4{seed, 0.0f, 0.0f, 0.0f};
    float s[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = seed * 0.01f + 0.003f * (float)(lane + i);
    const float a = 1.0e-3f * seed * (float)(lane + 1), bv = 1.0e-3f * seed;
    for (long long r = 0; r < reps; ++r) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[i], 0, 0, 0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int i = 0; i < 8; ++i) s[i] = (i & 1) ? __builtin_amdgcn_cosf(s[i]) : __builtin_amdgcn_sinf(s[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) out += (acc[i][0] + acc[i][1]) + (acc[i][2] + acc[i][3]);
#pragma unroll
    for (int i = 0; i < 8; ++i) out += s[i];
  } else if constexpr (KIND == 3 || KIND == 4) {
    constexpr int NC = KIND == 3 ? 4 : 1;
    probe_f32x4 acc[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) acc[i] = probe_f32x4{seed, 0.0f, 0.0f, 0.0f};
    const float a = 1.0e-3f * seed * (float)(lane + 1), bv = 1.0e-3f * seed;
    for (long long r = 0; r < reps; ++r) {
#pragma unroll
      for (int u = 0; u < kProbeUnroll / NC; ++u) {
#pragma unroll
        for (int i = 0; i < NC; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[i], 0, 0, 0);
      }
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) out += (acc[i][0] + acc[i][1]) + (acc[i][2] + acc[i][3]);
  } else if constexpr (KIND == 5) {
    probe_f32x16 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][e] = e == 0 ? seed : 0.0f;
    }
    const float a = 1.0e-3f * seed * (float)(lane + 1), bv = 1.0e-3f * seed;
    for (long long r = 0; r < reps; ++r) {
#pragma unroll
      for (int u = 0; u < kProbeUnroll / 4; ++u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc[i], 0, 0, 0);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int e = 0; e < 16; ++e) out += acc[i][e];
    }
  } else {
    // a lane's pixel coordinate and sixteen trap records (a, g, w), as in the pixel pass; c (the
    // row constant) changes once per repetition, so every term is computed anew
    const float U = (float)(2 * lane - 63), U2 = U * U;
    float ga[kProbeUnroll], aa[kProbeUnroll], wa[4];
#pragma unroll
    for (int i = 0; i < kProbeUnroll; ++i) {
      ga[i] = 1.0e-5f * (float)(i + 1) * seed;
      aa[i] = 0.01f * (float)(i + 1) * seed;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) wa[i] = 1.0f + 0.1f * (float)i;
    float c = 0.25f * seed, sr[4] = {0.0f, 0.0f, 0.0f, 0.0f}, si[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (long long r = 0; r < reps; ++r) {
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u) {
        const float t = __builtin_fmaf(ga[u], U2, __builtin_fmaf(aa[u], U, c));
        sr[u & 3] = __builtin_fmaf(wa[u & 3], __builtin_amdgcn_cosf(t), sr[u & 3]);
        si[u & 3] = __builtin_fmaf(wa[u & 3], __builtin_amdgcn_sinf(t), si[u & 3]);
      }
      c += 1.0e-3f;
    }
    out = ((sr[0] + si[0]) + (sr[1] + si[1])) + ((sr[2] + si[2]) + (sr[3] + si[3]));
  }
  const unsigned long long c1 = shader_clock(), r1 = real_clock();
  sink[blockIdx.x * blockDim.x + threadIdx.x] = out;
  if (lane == 0) {
    // vector stores of the wave's four stamps
    stamps[4 * (size_t)wave + 0] = c0;
    stamps[4 * (size_t)wave + 1] = c1;
    stamps[4 * (size_t)wave + 2] = r0;
    stamps[4 * (size_t)wave + 3] = r1;
  }
}

// Device-to-device copy for the bandwidth probe: every thread moves four 16-byte words per step,
// all four loads issued before the stores.
__global__ void __launch_bounds__(256)
k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * 1024;
  size_t i = (size_t)blockIdx.x * 1024 + threadIdx.x;
  for (; i + 768 < n; i += stride) {
    const uint4 v0 = src[i], v1 = src[i + 256], v2 = src[i + 512], v3 = src[i + 768];
    dst[i] = v0;
    dst[i + 256] = v1;
    dst[i + 512] = v2;
    dst[i + 768] = v3;
  }
  for (; i < n; i += 256) dst[i] = src[i];
}

}  // namespace

hipError_t launch_probe_copy(hipStream_t s, const void* src, void* dst, size_t n16, int blocks) {
  if (n16 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError();
}

int probe_ops_per_rep(int kind) {
  switch (kind) {
    case 0: return 8 * kProbeUnroll;         // FMA
    case 1: return 8 * kProbeUnroll;         // sin / cos
    case 2: return kProbeUnroll;             // terms (4 FMA + sin + cos each; plus 1 add per repetition)
    case 3:                                  // FLOPs per lane: 2 x 16 x 16 x 4 per product over 64 lanes
    case 4: return kProbeUnroll * 32;
    case 5: return kProbeUnroll * 64;        // 2 x 32 x 32 x 2 per product over 64 lanes
    case 6: return kProbeUnroll * 32;        // FLOPs of the products (the sin/cos beside them not counted)
    default: return 0;
  }
}

hipError_t launch_probe(hipStream_t s, int kind, int blocks, int threads, long long reps, float seed, float* sink,
                        unsigned long long* stamps) {
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(threads), 0, s, reps, seed, sink, stamps); break;
    case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(threads), 0, s, reps, seed, sink, stamps); break;
    case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(threads), 0, s, reps, seed, sink, stamps); break;
    case 3: hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(threads), 0, s, reps, seed, sink, stamps); break;
    case 4: hipLaunchKernelGGL(k_probe<4>, dim3(blocks), dim3(threads), 0, s, reps, seed, sink, stamps); break;
    case 5: hipLaunchKernelGGL(k_probe<5>, dim3(blocks), dim3(threads), 0, s, reps, seed, sink, stamps); break;
    case 6: hipLaunchKernelGGL(k_probe<6>, dim3(blocks), dim3(threads), 0, s, reps, seed, sink, stamps); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace hot
