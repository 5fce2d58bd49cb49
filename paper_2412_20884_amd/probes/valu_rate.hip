// VALU issue-rate probe behind the pair kernel's VALU-bound roofline: eight independent chains
// per lane of v_fma_f32, v_sub_f32 and v_exp_f32 (each exp followed by a v_mul_f32), 32 blocks of
// four waves per CU, timed with HIP events; prints the cycles one wave instruction takes on a
// SIMD at 2.4 GHz.  Build and run:
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2412_20884_amd/probes/valu_rate.hip -o /tmp/valu_rate && /tmp/valu_rate
#include <hip/hip_runtime.h>
#include <cstdio>
constexpr int ITERS = 4096;
__global__ __launch_bounds__(256) void k_fma(float *out, float s) {
  float a[8];
  for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 1e-3f + j;
  for (int i = 0; i < ITERS; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = fmaf(a[j], s, 0.5f);
  }
  float t = 0; for (int j = 0; j < 8; ++j) t += a[j];
  out[blockIdx.x * 256 + threadIdx.x] = t;
}
__global__ __launch_bounds__(256) void k_sub(float *out, float s) {
  float a[8];
  for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 1e-3f + j;
  for (int i = 0; i < ITERS; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = s - a[j];
  }
  float t = 0; for (int j = 0; j < 8; ++j) t += a[j];
  out[blockIdx.x * 256 + threadIdx.x] = t;
}
__global__ __launch_bounds__(256) void k_exp(float *out, float s) {
  float a[8];
  for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 1e-6f - j * 1e-3f;
  for (int i = 0; i < ITERS; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = __builtin_amdgcn_exp2f(a[j]) * s;
  }
  float t = 0; for (int j = 0; j < 8; ++j) t += a[j];
  out[blockIdx.x * 256 + threadIdx.x] = t;
}
int main() {
  int cus = 0; hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
  int clk = 0; hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, 0);
  const int blocks = cus * 32;  // 8 waves per SIMD worth of blocks (4 waves each)
  float *out; hipMalloc(&out, sizeof(float) * blocks * 256);
  hipEvent_t e0, e1; hipEventCreate(&e0); hipEventCreate(&e1);
  struct K { const char *name; void (*f)(float *, float); int ops_per_iter; };
  // ops_per_iter counts the timed instruction (for k_exp: one exp and its mul as one unit)
  K ks[3] = {{"v_fma_f32", k_fma, 8}, {"v_sub_f32", k_sub, 8}, {"v_exp_f32 + v_mul_f32", k_exp, 8}};
  for (auto &k : ks) {
    hipLaunchKernelGGL(k.f, dim3(blocks), dim3(256), 0, 0, out, 0.999f);
    hipDeviceSynchronize();
    hipEventRecord(e0);
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k.f, dim3(blocks), dim3(256), 0, 0, out, 0.999f);
    hipEventRecord(e1); hipEventSynchronize(e1);
    float ms; hipEventElapsedTime(&ms, e0, e1);
    const double wave_instr = 5.0 * blocks * 4.0 * ITERS * k.ops_per_iter;  // 4 waves per block
    const double per_simd = wave_instr / (cus * 4.0);
    const double cycles = per_simd / (ms * 1e-3 * 2.4e9);
    printf("%-20s %8.3f ms  lane-ops/s %.3e  => %.2f wave-instructions per SIMD-cycle at 2.4 GHz "
           "(%.2f cycles each); device clock attr %d kHz, CUs %d\n", k.name, ms,
           wave_instr * 64 / (ms * 1e-3), cycles, 1.0 / cycles, clk, cus);
  }
  return 0;
}
