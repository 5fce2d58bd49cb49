// Issue-cost probe for gfx950: shader cycles per wave instruction for the VALU forms and the
// MFMA shape the pair kernels use, measured against the shader clock the chip actually runs at
// (clock64 ticks over wall_clock64 ticks of the 100 MHz reference, wave 0 of every block).
//
//   table 1: one instruction form on 8 independent chains per lane, W waves per SIMD
//   table 2: v_fma_f32 with 1, 2, 4 or 8 independent chains (latency against throughput)
//   table 3: 16 v_fma_f32 on 8 chains plus M v_mfma_f32_16x16x32_f16 per loop trip in the same
//            waves: the cycles each MFMA adds when the VALU is saturated
//
// Every block has 256 threads (one wave per SIMD); W blocks per CU give W waves per SIMD. Each
// thread writes its result once to out[blockIdx.x * 256 + threadIdx.x] (out holds
// kMaxW * CUs * 256 floats) and thread 0 writes two clock counts to ck[2 * blockIdx.x + 0..1].
// Build and run:
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2412_20884_amd/probes/issue_rate.hip -o /tmp/issue_rate && /tmp/issue_rate
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kIters = 2048;  // chain steps per thread: 8 * kIters
constexpr int kMaxW = 8;
constexpr int kMaxCus = 256;
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

enum Form { kFmaVVV, kFmaVSV, kFmaInline, kFmaLiteral, kSub, kMul, kExp2, kCvtPk, kForms };
const char *kFormName[kForms] = {"v_fma_f32 v,v,v", "v_fma_f32 v,s,v", "v_fma_f32 v,v,0.5",
                                 "v_fma_f32 v,v,lit", "v_sub_f32 v,v", "v_mul_f32 v,v",
                                 "v_exp_f32", "v_cvt_pkrtz_f16_f32"};

template <int F>
__device__ __forceinline__ float step(float a, float b, float c, float s) {
  if (F == kFmaVVV) return fmaf(a, b, c);
  if (F == kFmaVSV) return fmaf(a, s, c);  // s is a kernel argument: an SGPR operand
  if (F == kFmaInline) return fmaf(a, b, 0.5f);
  if (F == kFmaLiteral) return fmaf(a, b, 0.3f);
  if (F == kSub) return b - a;
  if (F == kMul) return a * b;
  if (F == kExp2) return __builtin_amdgcn_exp2f(-a);
  return __builtin_bit_cast(float, __builtin_amdgcn_cvt_pkrtz(a, b));
}

__device__ __forceinline__ void init(float *a, float *b, float *c, int n) {
  for (int j = 0; j < n; ++j) {
    a[j] = 0.25f + threadIdx.x * 1e-4f + j * 1e-2f;
    b[j] = 0.999f - threadIdx.x * 1e-7f * j;
    c[j] = 1e-3f * j + threadIdx.x * 1e-9f;
  }
}

__device__ __forceinline__ void finish(float t, float *out, unsigned long long *ck,
                                       unsigned long long c0, unsigned long long w0) {
  out[blockIdx.x * 256 + threadIdx.x] = t;
  if (threadIdx.x == 0) {
    ck[2 * blockIdx.x] = clock64() - c0;
    ck[2 * blockIdx.x + 1] = wall_clock64() - w0;
  }
}

template <int CH, int F>
__global__ __launch_bounds__(256) void chains(float *out, float s, unsigned long long *ck) {
  const unsigned long long c0 = clock64(), w0 = wall_clock64();
  float a[CH], b[CH], c[CH];
  init(a, b, c, CH);
  for (int i = 0; i < kIters * 8 / CH; ++i) {
#pragma unroll
    for (int j = 0; j < CH; ++j) a[j] = step<F>(a[j], b[j], c[j], s);
  }
  float t = 0.f;
#pragma unroll
  for (int j = 0; j < CH; ++j) t += a[j];
  finish(t, out, ck, c0, w0);
}

template <int M>
__global__ __launch_bounds__(256) void fma_mfma(float *out, float s, unsigned long long *ck) {
  const unsigned long long c0 = clock64(), w0 = wall_clock64();
  float a[8], b[8], c[8];
  init(a, b, c, 8);
  h8 x, y;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    x[q] = (_Float16)(1e-3f * (threadIdx.x & 7));
    y[q] = (_Float16)(1e-3f * q);
  }
  f4 z[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) z[q] = f4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < kIters / 2; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = fmaf(a[j], b[j], c[j]);
#pragma unroll
    for (int q = 0; q < M; ++q)
      z[q & 3] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, z[q & 3], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = fmaf(a[j], b[j], c[j]);
  }
  float t = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) t += a[j];
#pragma unroll
  for (int q = 0; q < 4; ++q) t += z[q][0] + z[q][1] + z[q][2] + z[q][3];
  finish(t, out, ck, c0, w0);
}

typedef void (*Kernel)(float *, float, unsigned long long *);
float *g_out;
unsigned long long *g_ck;
unsigned long long g_hck[2 * kMaxW * kMaxCus];
int g_cus;

// shader cycles per chain step and wave, at the measured clock; also returns that clock (MHz)
double cycles(Kernel k, int w, double *mhz) {
  const int blocks = g_cus * w;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, 0, g_out, 0.999f, g_ck);
  hipDeviceSynchronize();
  hipEventRecord(e0);
  for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, 0, g_out, 0.999f, g_ck);
  hipEventRecord(e1);
  hipEventSynchronize(e1);
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipMemcpy(g_hck, g_ck, sizeof(unsigned long long) * 2 * blocks, hipMemcpyDeviceToHost);
  double sc = 0, sw = 0;
  for (int b = 0; b < blocks; ++b) {
    sc += (double)g_hck[2 * b];
    sw += (double)g_hck[2 * b + 1];
  }
  const double hz = 1e8 * sc / sw;
  if (mhz) *mhz = hz * 1e-6;
  return ms * 1e-3 / 5 * hz / (w * 8.0 * kIters);
}

}  // namespace

int main() {
  hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, 0);
  if (g_cus > kMaxCus) return 1;
  hipMalloc(&g_out, sizeof(float) * kMaxW * g_cus * 256);
  hipMalloc(&g_ck, sizeof(unsigned long long) * 2 * kMaxW * g_cus);
  const int ws[4] = {1, 2, 4, 8};
  double mhz = 0.0;
  printf("CUs %d. Shader cycles per wave instruction (chain step), at the measured clock\n", g_cus);
  printf("table 1 (8 chains)        W=1     W=2     W=4     W=8   clock at W=8\n");
  const Kernel forms[kForms] = {chains<8, kFmaVVV>,    chains<8, kFmaVSV>, chains<8, kFmaInline>,
                                chains<8, kFmaLiteral>, chains<8, kSub>,    chains<8, kMul>,
                                chains<8, kExp2>,       chains<8, kCvtPk>};
  for (int f = 0; f < kForms; ++f) {
    double c[4];
    for (int q = 0; q < 4; ++q) c[q] = cycles(forms[f], ws[q], &mhz);
    printf("%-22s %7.2f %7.2f %7.2f %7.2f   %4.0f MHz\n", kFormName[f], c[0], c[1], c[2], c[3], mhz);
  }
  printf("table 2 (v_fma_f32 v,v,v) W=1     W=2     W=4     W=8\n");
  const Kernel ilp[4] = {chains<1, kFmaVVV>, chains<2, kFmaVVV>, chains<4, kFmaVVV>, chains<8, kFmaVVV>};
  for (int q = 0; q < 4; ++q) {
    double c[4];
    for (int r = 0; r < 4; ++r) c[r] = cycles(ilp[q], ws[r], nullptr);
    printf("%d chains %14s %7.2f %7.2f %7.2f %7.2f\n", 1 << q, "", c[0], c[1], c[2], c[3]);
  }
  printf("table 3 (16 fma + M mfma per trip, W=8): cycles per trip and added per MFMA\n");
  const Kernel mix[5] = {fma_mfma<0>, fma_mfma<1>, fma_mfma<2>, fma_mfma<4>, fma_mfma<8>};
  const int ms_[5] = {0, 1, 2, 4, 8};
  double base = 0.0;
  for (int q = 0; q < 5; ++q) {
    const double trip = 16.0 * cycles(mix[q], 8, &mhz);
    if (q == 0) base = trip;
    if (q == 0)
      printf("M=%d %28.1f   %4.0f MHz\n", ms_[q], trip, mhz);
    else
      printf("M=%d %28.1f   %6.1f per MFMA   %4.0f MHz\n", ms_[q], trip, (trip - base) / ms_[q], mhz);
  }
  hipFree(g_out);
  hipFree(g_ck);
  return 0;
}
