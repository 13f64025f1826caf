// Measured VALU issue rates of the current device (measurement hook).
//
// The fused leaf kernels are bound by plain vector arithmetic: FP32
// multiply-adds and adds (v_fma_f32 / v_add_f32, never the packed forms) and
// one transcendental per point and column (v_exp_f32, v_sin_f32, v_cos_f32).
// Their roofline needs the rate of each instruction class; these kernels
// measure it.  Every thread runs eight independent dependency chains of one
// instruction class, so the issue rate, not the latency, sets the time.
#include <hip/hip_runtime.h>

#include "qmc_internal.h"

namespace qmc {

constexpr int kProbeIters = 1024;
constexpr int kProbeChains = 8;

template <int KIND>
__global__ __launch_bounds__(256) void valu_probe_kernel(float *__restrict__ out, float a, float b) {
  float x[kProbeChains];
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) x[i] = (float)threadIdx.x * 1e-3f + (float)i * 0.1f;
  for (int it = 0; it < kProbeIters; ++it) {
#pragma unroll
    for (int i = 0; i < kProbeChains; ++i) {
      if (KIND == 0) x[i] = fmaf(x[i], a, b);                  // v_fma_f32
      if (KIND == 1) x[i] = __builtin_amdgcn_exp2f(x[i]) * a;  // v_exp_f32 (+ one v_mul_f32)
      if (KIND == 2) x[i] = __builtin_amdgcn_sinf(x[i]);       // v_sin_f32
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) s += x[i];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Matrix-core issue rate: four independent accumulators per wave, back to back.
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KIND>
__global__ __launch_bounds__(256) void mfma_probe_kernel(float *__restrict__ out, float a) {
  const float x = a + (float)threadIdx.x * 1e-6f;
  float s = 0.f;
  if (KIND == 0) {  // v_mfma_f32_32x32x2_f32: 4096 flops
    f32x16 c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = f32x16{0};
    for (int it = 0; it < kProbeIters / 4; ++it)
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, x, c[i], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) s += c[i][0];
  } else if (KIND == 1) {  // v_mfma_f32_16x16x4_f32: 2048 flops
    f32x4 c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = f32x4{0};
    for (int it = 0; it < kProbeIters / 4; ++it)
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, x, c[i], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) s += c[i][0];
  } else {  // v_mfma_f32_32x32x16_bf16: 32768 flops
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (__bf16)x;
    f32x16 c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = f32x16{0};
    for (int it = 0; it < kProbeIters / 4; ++it)
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(v, v, c[i], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) s += c[i][0];
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace qmc

namespace {

qmc_status probe_fail(hipError_t e, const char *what, float *buf, hipEvent_t e0, hipEvent_t e1) {
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) (void)hipFree(buf);
  return qmc::record_error(QMC_EDEVICE, "VALU probe, %s: %s", what, hipGetErrorString(e));
}

template <int KIND>
hipError_t probe_one(int blocks, float *buf, hipEvent_t e0, hipEvent_t e1, hipStream_t st, double *rate) {
  // one untimed launch, then three timed ones
  hipLaunchKernelGGL(qmc::valu_probe_kernel<KIND>, dim3(blocks), dim3(256), 0, st, buf, 0.999f, 1e-4f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
  for (int rep = 0; rep < 3; ++rep)
    hipLaunchKernelGGL(qmc::valu_probe_kernel<KIND>, dim3(blocks), dim3(256), 0, st, buf, 0.999f, 1e-4f);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
  if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
  float ms = 0.f;
  if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
  const double ops = 3.0 * blocks * 256.0 * qmc::kProbeIters * qmc::kProbeChains;
  *rate = ms > 0.f ? ops / (ms * 1e-3) : 0.0;
  return hipSuccess;
}

template <int KIND>
hipError_t probe_mfma(int blocks, float *buf, hipEvent_t e0, hipEvent_t e1, hipStream_t st, double *rate) {
  hipLaunchKernelGGL(qmc::mfma_probe_kernel<KIND>, dim3(blocks), dim3(256), 0, st, buf, 0.5f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
  for (int rep = 0; rep < 3; ++rep)
    hipLaunchKernelGGL(qmc::mfma_probe_kernel<KIND>, dim3(blocks), dim3(256), 0, st, buf, 0.5f);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
  if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
  float ms = 0.f;
  if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
  const double per = KIND == 0 ? 4096.0 : KIND == 1 ? 2048.0 : 32768.0;  // flops per instruction
  const double waves = blocks * 4.0;
  const double flops = 3.0 * waves * (qmc::kProbeIters / 4) * 4 * per;
  *rate = ms > 0.f ? flops / (ms * 1e-3) : 0.0;
  return hipSuccess;
}

}  // namespace

extern "C" qmc_status qmc_probe_mfma(double *f32_32x32x2, double *f32_16x16x4, double *bf16_32x32x16,
                                     void *stream) {
  if (!f32_32x32x2 || !f32_16x16x4 || !bf16_32x32x16) return qmc::record_error(QMC_EINVAL, "null output pointer");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return qmc::record_error(QMC_EDEVICE, "no usable HIP device");
  const int blocks = cus * 8;  // eight workgroups of four waves per compute unit
  hipStream_t st = (hipStream_t)stream;
  float *buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&buf, (size_t)blocks * 256 * sizeof(float))) != hipSuccess)
    return probe_fail(e, "hipMalloc", nullptr, nullptr, nullptr);
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    return probe_fail(e, "hipEventCreate", buf, e0, e1);
  if ((e = probe_mfma<0>(blocks, buf, e0, e1, st, f32_32x32x2)) != hipSuccess ||
      (e = probe_mfma<1>(blocks, buf, e0, e1, st, f32_16x16x4)) != hipSuccess ||
      (e = probe_mfma<2>(blocks, buf, e0, e1, st, bf16_32x32x16)) != hipSuccess)
    return probe_fail(e, "probe", buf, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  return QMC_OK;
}

extern "C" qmc_status qmc_probe_valu(double *fma_per_s, double *exp_per_s, double *sin_per_s, void *stream) {
  if (!fma_per_s || !exp_per_s || !sin_per_s) return qmc::record_error(QMC_EINVAL, "null output pointer");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return qmc::record_error(QMC_EDEVICE, "no usable HIP device");
  const int blocks = cus * 16;  // 16 workgroups of four waves per compute unit
  hipStream_t st = (hipStream_t)stream;
  float *buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&buf, (size_t)blocks * 256 * sizeof(float))) != hipSuccess)
    return probe_fail(e, "hipMalloc", nullptr, nullptr, nullptr);
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    return probe_fail(e, "hipEventCreate", buf, e0, e1);
  if ((e = probe_one<0>(blocks, buf, e0, e1, st, fma_per_s)) != hipSuccess ||
      (e = probe_one<1>(blocks, buf, e0, e1, st, exp_per_s)) != hipSuccess ||
      (e = probe_one<2>(blocks, buf, e0, e1, st, sin_per_s)) != hipSuccess)
    return probe_fail(e, "probe", buf, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  return QMC_OK;
}
