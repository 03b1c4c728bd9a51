// nb_step.hip -- kick-drift of the KDK leapfrog in FP64 (section 4.3: after
// the forces are written back the orbits are integrated; the paper does not
// name the integrator).  Optionally adds the pull of a fixed point mass at
// the origin (unsoftened).
#include "nb_internal.h"

namespace nb {
namespace {

__global__ void __launch_bounds__(256)
k_kick_drift(int64_t n, const float4* __restrict__ acc,
             double4* __restrict__ pos, double* __restrict__ vx,
             double* __restrict__ vy, double* __restrict__ vz, double dtk,
             double dtd, double gm_ext) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 a = acc[i];
  double4 p = pos[i];
  double gx = (double)a.x, gy = (double)a.y, gz = (double)a.z;
  // every operation rounded once, in the order written, so that the FP64
  // update matches a plain scalar evaluation bit for bit
  if (gm_ext != 0.0) {
    const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(p.x, p.x),
                                          __dmul_rn(p.y, p.y)),
                                __dmul_rn(p.z, p.z));
    const double r = __dsqrt_rn(r2);
    const double k = __ddiv_rn(gm_ext, __dmul_rn(r2, r));
    gx = __dsub_rn(gx, __dmul_rn(k, p.x));
    gy = __dsub_rn(gy, __dmul_rn(k, p.y));
    gz = __dsub_rn(gz, __dmul_rn(k, p.z));
  }
  const double ux = __dadd_rn(vx[i], __dmul_rn(gx, dtk));
  const double uy = __dadd_rn(vy[i], __dmul_rn(gy, dtk));
  const double uz = __dadd_rn(vz[i], __dmul_rn(gz, dtk));
  vx[i] = ux;
  vy[i] = uy;
  vz[i] = uz;
  p.x = __dadd_rn(p.x, __dmul_rn(ux, dtd));
  p.y = __dadd_rn(p.y, __dmul_rn(uy, dtd));
  p.z = __dadd_rn(p.z, __dmul_rn(uz, dtd));
  pos[i] = p;
}

}  // namespace

int launch_kick_drift(nb_ctx* c, double dt_kick, double dt_drift) {
  hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(c->n, 256)), dim3(256), 0,
                     c->stream, c->n, (const float4*)c->acc.p, c->pos.p,
                     c->vx.p, c->vy.p, c->vz.p, dt_kick, dt_drift,
                     c->cfg.G * c->cfg.ext_mass);
  return hip_check(c, hipGetLastError(), "kick-drift launch");
}

}  // namespace nb

// ---------------------------------------------------------------------------
// Input packing and small fills.
namespace nb {
namespace {

__global__ void __launch_bounds__(256)
k_pack(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
       const double* __restrict__ z, const double* __restrict__ m,
       double4* __restrict__ pos, uint32_t* __restrict__ orig) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pos[i] = make_double4(x[i], y[i], z[i], m[i]);
  orig[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(256)
k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

int launch_pack(nb_ctx* c, const double* x, const double* y, const double* z,
                const double* m) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for(c->n, 256)), dim3(256), 0,
                     c->stream, c->n, x, y, z, m, c->pos.p, c->orig.p);
  return hip_check(c, hipGetLastError(), "pack launch");
}

int fill_u32(nb_ctx* c, uint32_t* p, int64_t n, uint32_t v) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0,
                     c->stream, p, n, v);
  return hip_check(c, hipGetLastError(), "fill launch");
}

}  // namespace nb
