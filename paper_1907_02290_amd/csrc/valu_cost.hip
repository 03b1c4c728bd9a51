// valu_cost.hip -- issue cost of the vector instructions the monopole force
// term is made of, measured on the device (a standalone program, not part of
// the library).
//
// Every kernel runs 8 independent dependency chains per lane at 8 waves per
// SIMD, long enough (tens of ms) for the clock to settle.  The shader clock
// is read with clock64() and the 100 MHz constant clock with
// wall_clock64() around each lane's loop, so costs are reported in actual
// shader cycles per wave64 instruction per SIMD as well as at the 2.4 GHz
// peak clock.  The last kernels evaluate the force kernel's monopole term
// (three offsets, r^2 + eps^2, one reciprocal square root, m/r, m/r^3, three
// acceleration FMAs and the potential) on j-data held in registers, the same
// term with a multiply in place of the reciprocal square root, and an rsq
// issued beside eight FMAs that do not depend on it (cycles per group).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#define CHECK(x)                                                            \
  do {                                                                      \
    hipError_t e_ = (x);                                                    \
    if (e_ != hipSuccess) {                                                 \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_),       \
                  __LINE__);                                                \
      return 1;                                                             \
    }                                                                       \
  } while (0)

namespace {

constexpr int kBlock = 256;

// records (shader cycles, constant-clock ticks) of lane 0 of each workgroup
__device__ __forceinline__ void stamp(unsigned long long* clk, int slot,
                                      unsigned long long c0,
                                      unsigned long long w0) {
  const unsigned long long c1 = clock64(), w1 = wall_clock64();
  if (threadIdx.x == 0) {
    clk[2 * slot] = c1 - c0;
    clk[2 * slot + 1] = w1 - w0;
  }
}

#define CHAINS(OP) OP(a0) OP(a1) OP(a2) OP(a3) OP(a4) OP(a5) OP(a6) OP(a7)

#define OP_KERNEL(name, OPMACRO)                                            \
  __global__ void __launch_bounds__(kBlock)                                 \
      name(int iters, float* sink, unsigned long long* clk) {               \
    float a0 = 1.0f + threadIdx.x * 1e-7f, a1 = a0 + 1e-3f,                 \
          a2 = a0 + 2e-3f, a3 = a0 + 3e-3f, a4 = a0 + 4e-3f,                \
          a5 = a0 + 5e-3f, a6 = a0 + 6e-3f, a7 = a0 + 7e-3f;                \
    const float b = 0.9999f + threadIdx.x * 1e-9f;                          \
    const float c = 1e-6f * (1 + threadIdx.x);                              \
    const unsigned long long c0 = clock64(), w0 = wall_clock64();           \
    for (int i = 0; i < iters; ++i) {                                       \
      _Pragma("unroll") for (int u = 0; u < 16; ++u) { CHAINS(OPMACRO) }    \
    }                                                                       \
    stamp(clk, blockIdx.x, c0, w0);                                         \
    if (a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7 == 12345.f) sink[0] = a0;     \
  }

#define OP_FMAC(a) \
  asm volatile("v_fmac_f32_e32 %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
#define OP_FMA3(a) \
  asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
#define OP_MUL(a) asm volatile("v_mul_f32_e32 %0, %1, %0" : "+v"(a) : "v"(b));
#define OP_SUB(a) asm volatile("v_sub_f32_e32 %0, %1, %0" : "+v"(a) : "v"(c));
#define OP_RSQ(a) asm volatile("v_rsq_f32_e32 %0, %0" : "+v"(a));

OP_KERNEL(k_fmac, OP_FMAC)
OP_KERNEL(k_fma3, OP_FMA3)
OP_KERNEL(k_mul, OP_MUL)
OP_KERNEL(k_sub, OP_SUB)
OP_KERNEL(k_rsq, OP_RSQ)

// The force kernel's monopole term; with TRANS false the reciprocal square
// root is replaced by a multiply, which leaves 14 plain FP32 operations and
// shows what the transcendental costs inside the term.
template <bool TRANS>
__device__ __forceinline__ void mono(const float4 j, float xi, float yi,
                                     float zi, float eps2, float& ax,
                                     float& ay, float& az, float& ph) {
  const float dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
  const float rinv = TRANS ? __builtin_amdgcn_rsqf(r2) : r2 * 0.5f;
  const float mr = j.w * rinv;
  const float mr3 = mr * rinv * rinv;
  ax = fmaf(mr3, dx, ax);
  ay = fmaf(mr3, dy, ay);
  az = fmaf(mr3, dz, az);
  ph -= mr;
}

// 64 terms per iteration on four j records read once from memory; the
// empty asm on x_i keeps the compiler from sharing work between repeats,
// so every term issues the force kernel's 13 FP32 operations and one rsq.
template <bool TRANS>
__global__ void __launch_bounds__(kBlock)
    k_mono(int iters, const float4* __restrict__ jd, float eps2, float* sink,
           unsigned long long* clk) {
  const float4 j0 = jd[0], j1 = jd[1], j2 = jd[2], j3 = jd[3];
  float xi = threadIdx.x * 1e-3f, yi = -(float)threadIdx.x * 2e-3f,
        zi = threadIdx.x * 5e-4f;
  float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
  const unsigned long long c0 = clock64(), w0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      asm volatile("" : "+v"(xi), "+v"(yi), "+v"(zi));
      mono<TRANS>(j0, xi, yi, zi, eps2, ax, ay, az, ph);
      mono<TRANS>(j1, xi, yi, zi, eps2, ax, ay, az, ph);
      mono<TRANS>(j2, xi, yi, zi, eps2, ax, ay, az, ph);
      mono<TRANS>(j3, xi, yi, zi, eps2, ax, ay, az, ph);
    }
  }
  stamp(clk, blockIdx.x, c0, w0);
  if (ax + ay + az + ph == 12345.f) sink[0] = ax;
}

// One rsq beside eight FMAs that do not depend on it.
__global__ void __launch_bounds__(kBlock)
    k_beside(int iters, float* sink, unsigned long long* clk) {
  float a0 = 1.0f + threadIdx.x * 1e-7f, a1 = a0 + 1e-3f, a2 = a0 + 2e-3f,
        a3 = a0 + 3e-3f, a4 = a0 + 4e-3f, a5 = a0 + 5e-3f, a6 = a0 + 6e-3f,
        a7 = a0 + 7e-3f, q0 = 1.0f + threadIdx.x * 1e-6f, q1 = q0 + 0.5f;
  const float b = 0.9999f + threadIdx.x * 1e-9f;
  const float c = 1e-6f * (1 + threadIdx.x);
  const unsigned long long c0 = clock64(), w0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      asm volatile("v_rsq_f32_e32 %0, %0" : "+v"(q0));
      CHAINS(OP_FMAC)
      asm volatile("v_rsq_f32_e32 %0, %0" : "+v"(q1));
      CHAINS(OP_FMAC)
    }
  }
  stamp(clk, blockIdx.x, c0, w0);
  if (a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7 + q0 + q1 == 12345.f)
    sink[0] = a0;
}

}  // namespace

int main() {
  int dev = 0, cus = 0, wall_khz = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              dev));
  CHECK(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate,
                              dev));
  const int simds = 4 * cus;
  const int nblk = 2 * simds;  // 8 waves of 64 lanes per SIMD
  float* sink = nullptr;
  float4* jd = nullptr;
  unsigned long long* clk = nullptr;
  CHECK(hipMalloc(&sink, sizeof(float)));
  CHECK(hipMalloc(&jd, 4 * sizeof(float4)));
  CHECK(hipMalloc(&clk, 2 * sizeof(unsigned long long) * nblk));
  const float4 hj[4] = {{0.1f, 0.2f, 0.3f, 1e-3f},
                        {-0.2f, 0.1f, 0.05f, 2e-3f},
                        {0.3f, -0.1f, 0.2f, 1e-3f},
                        {0.05f, 0.3f, -0.2f, 3e-3f}};
  CHECK(hipMemcpy(jd, hj, sizeof(hj), hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  std::vector<unsigned long long> h(2 * nblk);
  std::printf("%d CUs, %d SIMDs, %d waves of 64 lanes per SIMD\n", cus,
              simds, nblk * (kBlock / 64) / simds);
  std::printf("%-28s %9s %9s %14s %14s\n", "instruction or group", "ms",
              "clock GHz", "cycles", "at 2.4 GHz");

  struct Op {
    const char* name;
    void (*k)(int, float*, unsigned long long*);
  } ops[] = {{"v_fmac_f32 (VOP2)", k_fmac}, {"v_fma_f32 (VOP3)", k_fma3},
             {"v_mul_f32", k_mul},          {"v_sub_f32", k_sub},
             {"v_rsq_f32", k_rsq}};
  const char* mix_names[] = {"monopole term", "term, multiply for rsq",
                             "rsq + 8 independent FMAs"};
  for (int pass = -1; pass < 8; ++pass) {
    const bool warm = pass < 0;
    const int kind = warm ? 0 : pass;
    const int iters = warm ? 2000 : (kind == 4 ? 12000 : 40000);
    CHECK(hipEventRecord(e0));
    if (kind < 5)
      hipLaunchKernelGGL(ops[kind].k, dim3(nblk), dim3(kBlock), 0, 0, iters,
                         sink, clk);
    else if (kind == 5)
      hipLaunchKernelGGL(k_mono<true>, dim3(nblk), dim3(kBlock), 0, 0,
                         iters / 4, jd, 1e-4f, sink, clk);
    else if (kind == 6)
      hipLaunchKernelGGL(k_mono<false>, dim3(nblk), dim3(kBlock), 0, 0,
                         iters / 4, jd, 1e-4f, sink, clk);
    else
      hipLaunchKernelGGL(k_beside, dim3(nblk), dim3(kBlock), 0, 0, iters / 2,
                         sink, clk);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (warm) continue;
    CHECK(hipMemcpy(h.data(), clk, h.size() * sizeof(unsigned long long),
                    hipMemcpyDeviceToHost));
    std::vector<double> ghz(nblk);
    for (int b = 0; b < nblk; ++b)
      ghz[b] = (double)h[2 * b] /
               ((double)h[2 * b + 1] / (wall_khz * 1e3)) / 1e9;
    std::sort(ghz.begin(), ghz.end());
    const double f = ghz[nblk / 2];
    const double waves = (double)nblk * (kBlock / 64);
    if (kind < 5) {
      const double per_simd = (double)iters * 16 * 8 * waves / simds;
      std::printf("%-28s %9.3f %9.3f %14.2f %14.2f\n", ops[kind].name, ms, f,
                  ms * 1e-3 * f * 1e9 / per_simd,
                  ms * 1e-3 * 2.4e9 / per_simd);
    } else if (kind < 7) {
      // one wave's term covers 64 lane interactions
      const double inter = (double)(iters / 4) * 64 * waves * 64;
      const double per_simd = inter / 64 / simds;
      std::printf("%-28s %9.3f %9.3f %14.2f %14.2f   %.3e terms/s\n",
                  mix_names[kind - 5], ms, f, ms * 1e-3 * f * 1e9 / per_simd,
                  ms * 1e-3 * 2.4e9 / per_simd, inter / (ms * 1e-3));
    } else {
      const double per_simd = (double)(iters / 2) * 16 * waves / simds;
      std::printf("%-28s %9.3f %9.3f %14.2f %14.2f\n", mix_names[2], ms, f,
                  ms * 1e-3 * f * 1e9 / per_simd,
                  ms * 1e-3 * 2.4e9 / per_simd);
    }
  }
  CHECK(hipFree(sink));
  CHECK(hipFree(jd));
  CHECK(hipFree(clk));
  return 0;
}
