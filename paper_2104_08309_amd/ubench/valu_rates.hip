// Vector-ALU issue rates of gfx950 for the instruction classes of the face
// terms: the measured basis of the ALU ceiling of the FP32C kernels.
//
// Each kernel runs kChains independent dependency chains per thread over
// `iters` iterations, 8 wavefronts per SIMD (a block of 256 per CU slot, 8 x
// the CU count blocks), so every SIMD always has an independent instruction to
// issue and only the issue rate of the class limits the loop. The shader clock
// is measured beside the 100 MHz constant clock (clock64 over wall_clock64) for
// each kernel, since it drops under load. Output per class: the per-SIMD cycles
// one wave64 instruction occupies at the measured clock, lane operations per CU
// per cycle at that clock and at the nominal 2.4 GHz. Built with the library's
// flags (packed FP32 disabled), so each statement is one unpacked instruction.
// The last two classes issue the same sines and FMAs with the sines in one run or spread out (held in
// place by scheduling barriers): the difference is the cost of switching between the transcendental
// unit and ordinary vector instructions.
//
// Usage: valu_rates [iters]   (default 4096; prints one line per class)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK_HIP(x)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                                        \
    }                                                                                      \
  } while (0)

constexpr int kChains = 16;
constexpr int kBlock = 256;

enum Op {
  kFmac = 0,     // v_fmac_f32: a = b * c + a, all operands in VGPRs
  kMul,          // v_mul_f32
  kAdd,          // v_add_f32
  kFmaSgpr,      // v_fma_f32 with a wave-uniform (SGPR) operand
  kFmaVop3,      // v_fma_f32 (VOP3 encoding: destination not the addend), all operands in VGPRs
  kFmacSgpr,     // v_fmac_f32 (VOP2) with its first source a wave-uniform (SGPR) value
  kFmaak,        // v_fmaak_f32 (VOP2 with a literal addend)
  kMulNeg,       // v_mul_f32 in its VOP3 encoding with a negated source
  kFmaNegInl,    // v_fma_f32 (VOP3) with an inline constant and a negated source
  kSin,          // v_sin_f32 (argument in turns)
  kCos,          // v_cos_f32
  kRcp,          // v_rcp_f32
  kMix1to15,     // one v_sin_f32 per 15 v_fmac_f32, on separate chains
  kMix1to13,     // one v_sin_f32 per 13 v_fmac_f32 (the forward's share of transcendentals)
  kRun6,         // 6 v_sin_f32 in one run, then 90 v_fmac_f32 (scheduling barrier between)
  kSpread6,      // 6 x (1 v_sin_f32 + 15 v_fmac_f32), each group fenced by a scheduling barrier
  kOpsF32
};

// Instructions per chain-iteration of each class, counted per thread.
__host__ __device__ constexpr int ops_per_iter(int op) {
  return op == kMix1to15 ? kChains : op == kMix1to13 ? kChains - 2 : (op == kRun6 || op == kSpread6) ? 96 : kChains;
}

// The switch between the transcendental unit and ordinary vector instructions: the same 6 sines and 90
// FMAs per iteration (6 sine chains, 10 FMA chains), the sines in one run or spread one per 15 FMAs.
template <int OP>
__global__ __launch_bounds__(kBlock) void mix_kernel(float* out, unsigned long long* clk, int iters, float) {
  float t[6], a[10], b[10], c[10];
#pragma unroll
  for (int j = 0; j < 6; ++j) t[j] = 1e-3f * (float)(threadIdx.x + j) + 0.1f;
#pragma unroll
  for (int j = 0; j < 10; ++j) {
    a[j] = 1e-3f * (float)(threadIdx.x + j) + 0.1f;
    b[j] = 0.999f - 1e-5f * (float)(threadIdx.x + j);
    c[j] = 1e-4f * (float)(j + (threadIdx.x & 3));
  }
  const unsigned long long t0 = clock64(), w0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
    if (OP == kRun6) {
#pragma unroll
      for (int j = 0; j < 6; ++j) t[j] = __builtin_amdgcn_sinf(t[j]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 9; ++r)
#pragma unroll
        for (int j = 0; j < 10; ++j) a[j] = fmaf(b[j], c[j], a[j]);
    } else {
#pragma unroll
      for (int g = 0; g < 6; ++g) {
        t[g] = __builtin_amdgcn_sinf(t[g]);
#pragma unroll
        for (int j = 0; j < 15; ++j) {
          const int q = (g * 15 + j) % 10;
          a[q] = fmaf(b[q], c[q], a[q]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  const unsigned long long t1 = clock64(), w1 = wall_clock64();
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 6; ++j) s += t[j];
#pragma unroll
  for (int j = 0; j < 10; ++j) s += a[j];
  out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = w1 - w0;
  }
}

template <int OP>
__global__ __launch_bounds__(kBlock) void f32_kernel(float* out, unsigned long long* clk, int iters, float s1) {
  float a[kChains], b[kChains], c[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    a[j] = 1e-3f * (float)(threadIdx.x + j) + 0.1f;
    b[j] = 0.999f - 1e-5f * (float)(threadIdx.x + j);
    c[j] = 1e-4f * (float)(j + (threadIdx.x & 3));
  }
  const unsigned long long t0 = clock64(), w0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      if (OP == kFmac) a[j] = fmaf(b[j], c[j], a[j]);
      if (OP == kMul) a[j] = a[j] * b[j];
      if (OP == kAdd) a[j] = a[j] + c[j];
      if (OP == kFmaSgpr) a[j] = fmaf(a[j], b[j], s1);
      if (OP == kFmaVop3) a[j] = fmaf(a[j], b[j], c[j]);
      if (OP == kFmacSgpr) a[j] = fmaf(s1, b[j], a[j]);
      if (OP == kFmaak) a[j] = fmaf(a[j], b[j], 0.1234567f);
      if (OP == kMulNeg) a[j] = (-a[j]) * b[j];
      if (OP == kFmaNegInl) a[j] = fmaf(-2.0f, a[j], -c[j]);
      if (OP == kSin) a[j] = __builtin_amdgcn_sinf(a[j]);
      if (OP == kCos) a[j] = __builtin_amdgcn_cosf(a[j]);
      if (OP == kRcp) a[j] = __builtin_amdgcn_rcpf(a[j]);
      if (OP == kMix1to15) a[j] = j == 0 ? __builtin_amdgcn_sinf(a[j]) : fmaf(b[j], c[j], a[j]);
      if (OP == kMix1to13) {
        if (j == 0) a[j] = __builtin_amdgcn_sinf(a[j]);
        else if (j < kChains - 2) a[j] = fmaf(b[j], c[j], a[j]);
      }
    }
  }
  const unsigned long long t1 = clock64(), w1 = wall_clock64();
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += a[j];
  out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;  // keeps every chain live
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = w1 - w0;
  }
}

enum Op64 { kFma64 = 0, kAdd64, kOps64 };

template <int OP>
__global__ __launch_bounds__(kBlock) void f64_kernel(float* out, unsigned long long* clk, int iters, float) {
  constexpr int n = kChains / 2;
  double a[n], b[n], c[n];
#pragma unroll
  for (int j = 0; j < n; ++j) {
    a[j] = 1e-3 * (double)(threadIdx.x + j) + 0.1;
    b[j] = 0.999 - 1e-5 * (double)(threadIdx.x + j);
    c[j] = 1e-4 * (double)(j + (threadIdx.x & 3));
  }
  const unsigned long long t0 = clock64(), w0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < n; ++j) {
      if (OP == kFma64) a[j] = fma(b[j], c[j], a[j]);
      if (OP == kAdd64) a[j] = a[j] + c[j];
    }
  }
  const unsigned long long t1 = clock64(), w1 = wall_clock64();
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < n; ++j) s += a[j];
  out[(size_t)blockIdx.x * kBlock + threadIdx.x] = (float)s;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = w1 - w0;
  }
}

using Kernel = void (*)(float*, unsigned long long*, int, float);

struct Device {
  int cus = 0;
  int blocks = 0;
  float* out = nullptr;
  unsigned long long* dclk = nullptr;
  unsigned long long* hclk = nullptr;
};

// Best of 5 timed launches after one warm-up; the clock from the last launch's counters.
void run(const Device& d, const char* name, Kernel k, int iters, double ops_per_thread_iter) {
  hipEvent_t e0, e1;
  CHECK_HIP(hipEventCreate(&e0));
  CHECK_HIP(hipEventCreate(&e1));
  k<<<d.blocks, kBlock>>>(d.out, d.dclk, iters, 0.5f);
  CHECK_HIP(hipGetLastError());
  CHECK_HIP(hipDeviceSynchronize());
  float best = 1e30f;
  for (int r = 0; r < 5; ++r) {
    CHECK_HIP(hipEventRecord(e0));
    k<<<d.blocks, kBlock>>>(d.out, d.dclk, iters, 0.5f);
    CHECK_HIP(hipEventRecord(e1));
    CHECK_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) best = ms;
  }
  CHECK_HIP(hipMemcpy(d.hclk, d.dclk, sizeof(unsigned long long) * 2 * d.blocks, hipMemcpyDeviceToHost));
  double cyc = 0.0, wall = 0.0;
  for (int b = 0; b < d.blocks; ++b) {
    cyc += (double)d.hclk[2 * b];
    wall += (double)d.hclk[2 * b + 1];
  }
  const double ghz = 0.1 * cyc / wall;  // wall_clock64 runs at 100 MHz
  const double lane_ops = (double)d.blocks * kBlock * iters * ops_per_thread_iter;
  const double per_cu_cycle = lane_ops / ((double)best * 1e-3 * ghz * 1e9 * d.cus);
  const double per_cu_nominal = lane_ops / ((double)best * 1e-3 * 2.4e9 * d.cus);
  // a CU has 4 SIMDs; one wave64 instruction is 64 lane operations
  std::printf("%-34s %9.4f ms  clock %5.3f GHz  %6.2f SIMD-cycles/wave-instr  %7.2f lane-ops/CU/cycle  "
              "%7.2f at 2.4 GHz\n",
              name, best, ghz, 4.0 * 64.0 / per_cu_cycle, per_cu_cycle, per_cu_nominal);
  CHECK_HIP(hipEventDestroy(e0));
  CHECK_HIP(hipEventDestroy(e1));
}

int main(int argc, char** argv) {
  const int iters = argc > 1 ? std::atoi(argv[1]) : 4096;
  if (iters <= 0 || iters > (1 << 20)) {
    std::fprintf(stderr, "iters must be in 1 .. 2^20\n");
    return 2;
  }
  hipDeviceProp_t p;
  CHECK_HIP(hipGetDeviceProperties(&p, 0));
  Device d;
  d.cus = p.multiProcessorCount;
  d.blocks = d.cus * 8;  // 8 blocks of 4 wavefronts per CU: 8 wavefronts per SIMD
  CHECK_HIP(hipMalloc(&d.out, sizeof(float) * (size_t)d.blocks * kBlock));
  CHECK_HIP(hipMalloc(&d.dclk, sizeof(unsigned long long) * 2 * d.blocks));
  d.hclk = static_cast<unsigned long long*>(std::malloc(sizeof(unsigned long long) * 2 * d.blocks));
  if (!d.hclk) return 1;
  std::printf("device %s, %d CUs; %d blocks of %d, %d independent chains per thread, %d iterations\n",
              p.gcnArchName, d.cus, d.blocks, kBlock, kChains, iters);
  run(d, "v_fmac_f32 (VGPR operands)", f32_kernel<kFmac>, iters, ops_per_iter(kFmac));
  run(d, "v_mul_f32", f32_kernel<kMul>, iters, ops_per_iter(kMul));
  run(d, "v_add_f32", f32_kernel<kAdd>, iters, ops_per_iter(kAdd));
  run(d, "v_fma_f32 (one SGPR operand)", f32_kernel<kFmaSgpr>, iters, ops_per_iter(kFmaSgpr));
  run(d, "v_fma_f32 (VOP3, VGPR operands)", f32_kernel<kFmaVop3>, iters, ops_per_iter(kFmaVop3));
  run(d, "v_fmac_f32 (SGPR first source)", f32_kernel<kFmacSgpr>, iters, ops_per_iter(kFmacSgpr));
  run(d, "v_fmaak_f32 (literal addend)", f32_kernel<kFmaak>, iters, ops_per_iter(kFmaak));
  run(d, "v_mul_f32_e64 (negated source)", f32_kernel<kMulNeg>, iters, ops_per_iter(kMulNeg));
  run(d, "v_fma_f32 (inline const, neg)", f32_kernel<kFmaNegInl>, iters, ops_per_iter(kFmaNegInl));
  run(d, "v_sin_f32", f32_kernel<kSin>, iters, ops_per_iter(kSin));
  run(d, "v_cos_f32", f32_kernel<kCos>, iters, ops_per_iter(kCos));
  run(d, "v_rcp_f32", f32_kernel<kRcp>, iters, ops_per_iter(kRcp));
  run(d, "1 v_sin_f32 : 15 v_fmac_f32", f32_kernel<kMix1to15>, iters, ops_per_iter(kMix1to15));
  run(d, "1 v_sin_f32 : 13 v_fmac_f32", f32_kernel<kMix1to13>, iters, ops_per_iter(kMix1to13));
  run(d, "6 v_sin_f32 in one run + 90 fmac", mix_kernel<kRun6>, iters, ops_per_iter(kRun6));
  run(d, "6 x (1 v_sin_f32 + 15 fmac)", mix_kernel<kSpread6>, iters, ops_per_iter(kSpread6));
  run(d, "v_fma_f64", f64_kernel<kFma64>, iters, kChains / 2);
  run(d, "v_add_f64", f64_kernel<kAdd64>, iters, kChains / 2);
  CHECK_HIP(hipFree(d.out));
  CHECK_HIP(hipFree(d.dclk));
  std::free(d.hclk);
  return 0;
}
