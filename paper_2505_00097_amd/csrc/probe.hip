// probe.hip -- measured machine peaks for the roofline: FP64 FMA throughput
// and streaming HBM bandwidth on the current device.
#include "bhah_internal.h"

namespace bhah {

// Independent FMA chains per thread (enough to hide the FP64 pipeline
// latency); the result is stored so nothing is optimised away.
constexpr int FMA_CHAINS = 8;
constexpr int FMA_ITERS = 4096;

__global__ void __launch_bounds__(256) k_fma_chain(double* __restrict__ out, double a, double b) {
  double acc[FMA_CHAINS];
#pragma unroll
  for (int c = 0; c < FMA_CHAINS; c++) acc[c] = (double)(threadIdx.x + c) * 1e-3;
  for (int it = 0; it < FMA_ITERS; it++) {
#pragma unroll
    for (int c = 0; c < FMA_CHAINS; c++) acc[c] = fma(acc[c], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < FMA_CHAINS; c++) s += acc[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// a = b + s c, 16 bytes per thread per array (two doubles)
__global__ void __launch_bounds__(256) k_triad(double2* __restrict__ a, const double2* __restrict__ b,
                                               const double2* __restrict__ c, double s, long long n2) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2; i += stride) {
    const double2 x = b[i], z = c[i];
    a[i] = double2{x.x + s * z.x, x.y + s * z.y};
  }
}

}  // namespace bhah

using namespace bhah;

extern "C" {

int bhah_probe_peaks(double* fp64_tflops, double* hbm_gbps, void* stream) {
  if (!fp64_tflops || !hbm_gbps) return fail(BHAH_EINVAL, "bhah_probe_peaks: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, cus = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (!rc) rc = check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  if (rc) return rc;
  const int fma_blocks = 64 * cus;  // 16 waves per CU
  const long long n2 = 1LL << 27;   // 2^27 double2 = 2 GiB per array
  double *out = nullptr, *a = nullptr, *b = nullptr, *c = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&out, sizeof(double) * 256 * (size_t)fma_blocks);
  if (e == hipSuccess) e = hipMalloc((void**)&a, sizeof(double2) * (size_t)n2);
  if (e == hipSuccess) e = hipMalloc((void**)&b, sizeof(double2) * (size_t)n2);
  if (e == hipSuccess) e = hipMalloc((void**)&c, sizeof(double2) * (size_t)n2);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemsetAsync(b, 0, sizeof(double2) * (size_t)n2, s);
  if (e == hipSuccess) e = hipMemsetAsync(c, 0, sizeof(double2) * (size_t)n2, s);
  float ms_fma = 0.f, ms_triad = 0.f;
  const int reps = 5;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fma_chain, dim3(fma_blocks), dim3(256), 0, s, out, 0.999, 1e-6);
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; r++)
      hipLaunchKernelGGL(k_fma_chain, dim3(fma_blocks), dim3(256), 0, s, out, 0.999, 1e-6);
    (void)hipEventRecord(e1, s);
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_fma, e0, e1);
  }
  if (e == hipSuccess) {
    const int tb = 16 * cus;
    hipLaunchKernelGGL(k_triad, dim3(tb), dim3(256), 0, s, (double2*)a, (const double2*)b, (const double2*)c, 0.5, n2);
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; r++)
      hipLaunchKernelGGL(k_triad, dim3(tb), dim3(256), 0, s, (double2*)a, (const double2*)b, (const double2*)c, 0.5,
                         n2);
    (void)hipEventRecord(e1, s);
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms_triad, e0, e1);
  }
  if (e == hipSuccess) e = hipGetLastError();
  for (double* p : {out, a, b, c})
    if (p) (void)hipFree(p);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return check_hip(e, "bhah_probe_peaks");
  const double flops = 2.0 * FMA_CHAINS * FMA_ITERS * 256.0 * fma_blocks * reps;
  *fp64_tflops = flops / (ms_fma * 1e-3) / 1e12;
  const double bytes = 3.0 * sizeof(double2) * (double)n2 * reps;
  *hbm_gbps = bytes / (ms_triad * 1e-3) / 1e9;
  return BHAH_OK;
}

}  // extern "C"
