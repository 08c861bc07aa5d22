// Issue-rate microbenchmark of the VALU operations the a/j/s kernels are
// made of, on the current GPU: FP64 FMA, FP64 reciprocal-square-root
// estimate, FP32 FMA, FP32 estimate, an FP64->FP32->FP64 conversion pair
// (with an add so the pair cannot fold away), and 1 rsq : 3 FMA. Each thread
// runs 8 independent dependency chains; one store per thread at the end.
// It gives the practical per-CU rates against which the kernels' issue
// ceilings are judged (the nominal peak assumes the 2.4 GHz peak clock).
#include <hip/hip_runtime.h>
#include <cstdio>
constexpr int ITER = 4096;
#define CHAINS 8
__global__ void k_fma64(double* out, double a, double b) {
  double x[CHAINS]; for (int c = 0; c < CHAINS; ++c) x[c] = threadIdx.x * 1e-3 + c;
  for (int i = 0; i < ITER; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = fma(x[c], a, b);
  double s = 0; for (int c = 0; c < CHAINS; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void k_rsq64(double* out) {
  double x[CHAINS]; for (int c = 0; c < CHAINS; ++c) x[c] = 1.5 + threadIdx.x * 1e-3 + c;
  for (int i = 0; i < ITER; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = __builtin_amdgcn_rsq(x[c]);
  double s = 0; for (int c = 0; c < CHAINS; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void k_fma32(double* out, float a, float b) {
  float x[CHAINS]; for (int c = 0; c < CHAINS; ++c) x[c] = threadIdx.x * 1e-3f + c;
  for (int i = 0; i < ITER; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = fmaf(x[c], a, b);
  float s = 0; for (int c = 0; c < CHAINS; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void k_rsq32(double* out) {
  float x[CHAINS]; for (int c = 0; c < CHAINS; ++c) x[c] = 1.5f + threadIdx.x * 1e-3f + c;
  for (int i = 0; i < ITER; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = __builtin_amdgcn_rsqf(x[c]);
  float s = 0; for (int c = 0; c < CHAINS; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void k_cvt(double* out) {
  double x[CHAINS]; for (int c = 0; c < CHAINS; ++c) x[c] = 1.5 + threadIdx.x * 1e-3 + c;
  for (int i = 0; i < ITER; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = (double)((float)x[c]) + 1e-3;
  double s = 0; for (int c = 0; c < CHAINS; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void k_mix(double* out, double a, double b) {  // 3 fma64 : 1 rsq64
  double x[CHAINS]; for (int c = 0; c < CHAINS; ++c) x[c] = 1.5 + threadIdx.x * 1e-3 + c;
  for (int i = 0; i < ITER; ++i)
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) { double y = __builtin_amdgcn_rsq(x[c]); x[c] = fma(fma(fma(y, a, b), a, b), a, 1.5); }
  double s = 0; for (int c = 0; c < CHAINS; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
int main() {
  printf("# ops per CU per clock are computed at 2.4 GHz with 256 CUs; a full-rate FP64 FMA\n"
         "# would read 64 (one wave64 FMA per SIMD every 4 clocks)\n");
  const int blocks = 256 * 16, threads = 256;
  double* out; hipMalloc(&out, sizeof(double) * blocks * threads);
  hipEvent_t e0, e1; hipEventCreate(&e0); hipEventCreate(&e1);
  const double ops = (double)blocks * threads * CHAINS * ITER;
  for (int k = 0; k < 6; ++k) {
    for (int rep = 0; rep < 2; ++rep) {
      hipEventRecord(e0, 0);
      switch (k) {
        case 0: hipLaunchKernelGGL(k_fma64, dim3(blocks), dim3(threads), 0, 0, out, 0.999999, 1e-7); break;
        case 1: hipLaunchKernelGGL(k_rsq64, dim3(blocks), dim3(threads), 0, 0, out); break;
        case 2: hipLaunchKernelGGL(k_fma32, dim3(blocks), dim3(threads), 0, 0, out, 0.999999f, 1e-7f); break;
        case 3: hipLaunchKernelGGL(k_rsq32, dim3(blocks), dim3(threads), 0, 0, out); break;
        case 4: hipLaunchKernelGGL(k_cvt, dim3(blocks), dim3(threads), 0, 0, out); break;
        case 5: hipLaunchKernelGGL(k_mix, dim3(blocks), dim3(threads), 0, 0, out, 0.5, 0.25); break;
      }
      hipEventRecord(e1, 0); hipEventSynchronize(e1);
      float ms; hipEventElapsedTime(&ms, e0, e1);
      const char* nm[] = {"fma_f64", "rsq_f64", "fma_f32", "rsq_f32", "cvt pair + add_f64", "rsq_f64 + 3 fma_f64"};
      if (rep) printf("%-24s %8.3f ms  %.3e ops/s  = %.3f ops per CU per clock at 2.4 GHz\n", nm[k], ms, ops / (ms * 1e-3), ops / (ms * 1e-3) / 256 / 2.4e9);
    }
  }
  return 0;
}
