// Vector-unit rates of the GPU this runs on: the figures the benchmark's
// roofline peaks rest on.  Prints one JSON object.
//
//  * issue cycles per instruction of one wavefront running a chain of
//    dependent operations and, for FMA, four independent chains (core-clock
//    cycles from s_memtime): double FMA, single FMA, and the single-precision
//    sine and cosine of the transcendental unit;
//  * the core clock while every SIMD runs double FMAs (s_memtime cycles over
//    s_memrealtime ticks of the 100 MHz constant clock);
//  * whole-chip throughput with eight wavefronts per SIMD: double FMA
//    (TFLOP/s), single-precision sine plus cosine (Tops/s).
//
// Build: hipcc --offload-arch=gfx950 -O3 -o unit_rates unit_rates.hip
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kIters = 1024;

#define CHECK(x)                                                                         \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) {                                                              \
      std::fprintf(stderr, "unit_rates: %s: %s\n", #x, hipGetErrorString(e_));           \
      std::exit(1);                                                                      \
    }                                                                                    \
  } while (0)

// ---- one wavefront: cycles per instruction
__global__ void k_chain_f64(double a, double b, double* out, long long* cyc) {
  double x = a + threadIdx.x;
  const long long t0 = clock64();
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int j = 0; j < 16; ++j) x = fma(x, b, a);
  }
  const long long t1 = clock64();
  out[threadIdx.x] = x;
  if (threadIdx.x == 0) cyc[0] = t1 - t0;
}

__global__ void k_chain4_f64(double a, double b, double* out, long long* cyc) {
  double x0 = a + threadIdx.x, x1 = x0 + 1.0, x2 = x0 + 2.0, x3 = x0 + 3.0;
  const long long t0 = clock64();
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x0 = fma(x0, b, a); x1 = fma(x1, b, a); x2 = fma(x2, b, a); x3 = fma(x3, b, a);
    }
  }
  const long long t1 = clock64();
  out[threadIdx.x] = (x0 + x1) + (x2 + x3);
  if (threadIdx.x == 0) cyc[0] = t1 - t0;
}

__global__ void k_chain_f32(float a, float b, float* out, long long* cyc) {
  float x = a + threadIdx.x;
  const long long t0 = clock64();
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int j = 0; j < 16; ++j) x = fmaf(x, b, a);
  }
  const long long t1 = clock64();
  out[threadIdx.x] = x;
  if (threadIdx.x == 0) cyc[0] = t1 - t0;
}

__global__ void k_chain_sin(float a, float* out, long long* cyc) {
  float x = a + threadIdx.x * 1e-3f;
  const long long t0 = clock64();
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int j = 0; j < 16; ++j) x = __builtin_amdgcn_sinf(x);
  }
  const long long t1 = clock64();
  out[threadIdx.x] = x;
  if (threadIdx.x == 0) cyc[0] = t1 - t0;
}

__global__ void k_chain4_sincos(float a, float* out, long long* cyc) {
  float x0 = a + threadIdx.x * 1e-3f, x1 = x0 + 0.1f, x2 = x0 + 0.2f, x3 = x0 + 0.3f;
  const long long t0 = clock64();
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x0 = __builtin_amdgcn_sinf(x0); x1 = __builtin_amdgcn_cosf(x1);
      x2 = __builtin_amdgcn_sinf(x2); x3 = __builtin_amdgcn_cosf(x3);
    }
  }
  const long long t1 = clock64();
  out[threadIdx.x] = (x0 + x1) + (x2 + x3);
  if (threadIdx.x == 0) cyc[0] = t1 - t0;
}

// ---- whole chip: eight independent FMA chains per thread; the first
// thread of each block records core-clock and constant-clock spans
__global__ __launch_bounds__(256) void k_chip_f64(double a, double b, int iters, double* out, long long* clk) {
  double x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = a + threadIdx.x + c;
  const long long t0 = clock64();
  const long long r0 = __builtin_amdgcn_s_memrealtime();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = fma(x[c], b, a);
  }
  const long long t1 = clock64();
  const long long r1 = __builtin_amdgcn_s_memrealtime();
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[blockIdx.x * 256 + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = r1 - r0;
  }
}

__global__ __launch_bounds__(256) void k_chip_sincos(float a, int iters, float* out) {
  float x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = a + threadIdx.x * 1e-4f + c * 0.1f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; c += 2) {
      x[c] = __builtin_amdgcn_sinf(x[c]);
      x[c + 1] = __builtin_amdgcn_cosf(x[c + 1]);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

double one_wave(void (*launch)(long long*), long long* cyc_dev, double ops) {
  long long c = 0;
  launch(cyc_dev);     // first launch loads the code object
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  launch(cyc_dev);
  CHECK(hipGetLastError());
  CHECK(hipMemcpy(&c, cyc_dev, sizeof(c), hipMemcpyDeviceToHost));
  return (double)c / ops;
}

double* g_od;
float* g_of;

}  // namespace

int main() {
  int dev = 0, cus = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, dev));
  const int blocks = cus * 8;          // 256 threads each: eight wavefronts per SIMD
  long long* cyc = nullptr;
  long long* clk = nullptr;
  CHECK(hipMalloc((void**)&g_od, sizeof(double) * blocks * 256));
  CHECK(hipMalloc((void**)&g_of, sizeof(float) * blocks * 256));
  CHECK(hipMalloc((void**)&cyc, sizeof(long long)));
  CHECK(hipMalloc((void**)&clk, sizeof(long long) * 2 * blocks));
  const double ops = 16.0 * kIters;
  const double dep_f64 = one_wave([](long long* c) { hipLaunchKernelGGL(k_chain_f64, 1, 64, 0, 0, 0.5, 0.999, g_od, c); }, cyc, ops);
  const double ind_f64 = one_wave([](long long* c) { hipLaunchKernelGGL(k_chain4_f64, 1, 64, 0, 0, 0.5, 0.999, g_od, c); }, cyc, ops);
  const double dep_f32 = one_wave([](long long* c) { hipLaunchKernelGGL(k_chain_f32, 1, 64, 0, 0, 0.5f, 0.999f, g_of, c); }, cyc, ops);
  const double dep_sin = one_wave([](long long* c) { hipLaunchKernelGGL(k_chain_sin, 1, 64, 0, 0, 0.3f, g_of, c); }, cyc, ops);
  const double ind_sc = one_wave([](long long* c) { hipLaunchKernelGGL(k_chain4_sincos, 1, 64, 0, 0, 0.3f, g_of, c); }, cyc, ops);

  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const int it64 = 20000, itsc = 4000;
  hipLaunchKernelGGL(k_chip_f64, blocks, 256, 0, 0, 0.5, 0.999, 16, g_od, clk);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0, 0));
  hipLaunchKernelGGL(k_chip_f64, blocks, 256, 0, 0, 0.5, 0.999, it64, g_od, clk);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms64 = 0.0f;
  CHECK(hipEventElapsedTime(&ms64, e0, e1));
  long long* h = (long long*)std::malloc(sizeof(long long) * 2 * blocks);
  CHECK(hipMemcpy(h, clk, sizeof(long long) * 2 * blocks, hipMemcpyDeviceToHost));
  double core = 0.0, ref = 0.0;
  for (int i = 0; i < blocks; ++i) {
    core += (double)h[2 * i];
    ref += (double)h[2 * i + 1];
  }
  std::free(h);
  const double clock_ghz = core / ref * 0.1;    // constant clock: 100 MHz
  const double flops64 = 2.0 * 8.0 * it64 * (double)blocks * 256;
  hipLaunchKernelGGL(k_chip_sincos, blocks, 256, 0, 0, 0.3f, 16, g_of);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0, 0));
  hipLaunchKernelGGL(k_chip_sincos, blocks, 256, 0, 0, 0.3f, itsc, g_of);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float mssc = 0.0f;
  CHECK(hipEventElapsedTime(&mssc, e0, e1));
  const double opssc = 8.0 * itsc * (double)blocks * 256;
  std::printf("{\"device\": \"%s\", \"compute_units\": %d, "
              "\"cycles_per_instruction_one_wave\": {\"fma_f64_dependent\": %.2f, \"fma_f64_4_chains\": %.2f, "
              "\"fma_f32_dependent\": %.2f, \"sin_f32_dependent\": %.2f, \"sin_cos_f32_4_chains\": %.2f}, "
              "\"core_clock_ghz_under_fma_f64\": %.3f, \"chip_fma_f64_tflops\": %.2f, \"chip_sin_cos_f32_tops\": %.2f}\n",
              prop.gcnArchName, cus, dep_f64, ind_f64, dep_f32, dep_sin, ind_sc, clock_ghz,
              flops64 / (ms64 * 1e-3) / 1e12, opssc / (mssc * 1e-3) / 1e12);
  CHECK(hipFree(g_od));
  CHECK(hipFree(g_of));
  CHECK(hipFree(cyc));
  CHECK(hipFree(clk));
  return 0;
}
