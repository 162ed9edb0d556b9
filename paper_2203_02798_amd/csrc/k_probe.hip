// Ceiling probes: the attainable rates of the resources the path's kernels
// are bound by, measured on the device they run on, so that each
// kernel's roofline fraction can be stated against the datasheet peak and
// against what this device actually sustains.
//   copy      HBM: a grid-stride 16-byte copy (bytes read + bytes written);
//   mfma_f64  FP64 matrix cores: v_mfma_f64_16x16x4f64 on eight independent
//             register accumulators per wavefront (2048 flops each);
//   mfma_lowp the BF16 and FP8 matrix instructions of the Gaussian products
//             (v_mfma_f32_16x16x32_bf16, 16384 flops; the scaled e4m3
//             v_mfma_scale_f32_16x16x128_f8f6f4, 65536 flops), likewise;
//   valu_f32  vector ALU: eight independent v_fma_f32 chains per lane (one
//             lane-operation each; the library is compiled without packed
//             FP32 instructions).
// The arithmetic probes write one value per thread so the work is kept.
#include "internal.hpp"

namespace psk {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void k_probe_copy(const float4 *__restrict__ src,
                                                    float4 *__restrict__ dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_probe_mfma_f64(int64_t iters, double *__restrict__ out) {
  v4d acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
  const double a = 1.0 + threadIdx.x * 1e-3, b = 1.0 - threadIdx.x * 1e-3;
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_mfma_f32_16x16x32_bf16, 16384 flops each.
__global__ __launch_bounds__(256) void k_probe_mfma_bf16(int64_t iters, float *__restrict__ out) {
  v4f acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
  const __bf16 one = (__bf16)1.0f, sm = (__bf16)(threadIdx.x * 1e-3f);
  const v8bf a = {one, sm, one, sm, one, sm, one, sm};
  const v8bf b = {sm, one, sm, one, sm, one, sm, one};
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// v_mfma_scale_f32_16x16x128_f8f6f4 with both operands e4m3 and unit E8M0
// scales (the form the FP8 Gaussian product uses), 65536 flops each.
__global__ __launch_bounds__(256) void k_probe_mfma_fp8(int64_t iters, float *__restrict__ out) {
  v4f acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
  const int w = 0x38383838 ^ (int)(threadIdx.x & 1);  // e4m3 1.0, 1.125
  const v8i a = {w, w, w, w, w, w, w, w};
  const v8i b = {w, w, w, w, w, w, w, w};
  const int sc = 0x7f7f7f7f;  // E8M0 2^0
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
      acc[c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[c], 0, 0, 0, sc, 0, sc);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_valu_f32(int64_t iters, float *__restrict__ out) {
  float x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = 1.0f + (float)(threadIdx.x + c) * 1e-6f;
  const float a = 0.999999f, b = 1e-7f;
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = fmaf(x[c], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace
}  // namespace psk

using namespace psk;

extern "C" {

int psk_probe_copy(const void *src, void *dst, size_t bytes, void *stream) {
  if (!src || !dst) return fail(PSK_EINVAL, "src and dst must be non-NULL");
  if (bytes == 0 || bytes % 16 != 0) return fail(PSK_EINVAL, "bytes must be a positive multiple of 16");
  if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(PSK_EINVAL, "src and dst must be 16-byte aligned");
  const int64_t count = (int64_t)(bytes / 16);
  k_probe_copy<<<2048, 256, 0, (hipStream_t)stream>>>((const float4 *)src, (float4 *)dst, count);
  PSK_HIP_TRY(hipGetLastError());
  return PSK_OK;
}

int psk_probe_mfma_f64(int64_t iters, double *out, void *stream) {
  if (!out || iters < 1) return fail(PSK_EINVAL, "out must be non-NULL and iters >= 1");
  k_probe_mfma_f64<<<PSK_PROBE_BLOCKS, 256, 0, (hipStream_t)stream>>>(iters, out);
  PSK_HIP_TRY(hipGetLastError());
  return PSK_OK;
}

int psk_probe_mfma_lowp(int fmt, int64_t iters, float *out, void *stream) {
  if (!out || iters < 1) return fail(PSK_EINVAL, "out must be non-NULL and iters >= 1");
  if (fmt == PSK_PREC_BF16)
    k_probe_mfma_bf16<<<PSK_PROBE_BLOCKS, 256, 0, (hipStream_t)stream>>>(iters, out);
  else if (fmt == PSK_PREC_FP8)
    k_probe_mfma_fp8<<<PSK_PROBE_BLOCKS, 256, 0, (hipStream_t)stream>>>(iters, out);
  else
    return fail(PSK_EDTYPE, "fmt must be PSK_PREC_BF16 or PSK_PREC_FP8");
  PSK_HIP_TRY(hipGetLastError());
  return PSK_OK;
}

int psk_probe_valu_f32(int64_t iters, float *out, void *stream) {
  if (!out || iters < 1) return fail(PSK_EINVAL, "out must be non-NULL and iters >= 1");
  k_probe_valu_f32<<<PSK_PROBE_BLOCKS, 256, 0, (hipStream_t)stream>>>(iters, out);
  PSK_HIP_TRY(hipGetLastError());
  return PSK_OK;
}

}  // extern "C"
