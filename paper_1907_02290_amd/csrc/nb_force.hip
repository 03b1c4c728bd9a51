// nb_force.hip -- the multiwalk force kernel (section 3, Hamada et al.'s
// multiwalk; section 4.1, lists of indices into device-resident particle
// and cell arrays): one launch evaluates every group's list.
//
// Mapping on CDNA4 (wave64, LDS, 8 XCDs):
//  * one work item = one group, or a chunk of at most 64 of its particles;
//    one wavefront (a 64-thread workgroup) per work item;
//  * one i-particle per lane, as FP32 offsets from the group centre (the
//    FP64 subtraction is done once per particle and once per list entry);
//  * a group of n_i < 33 particles is replicated over r = 64 / n_i lane
//    slices; slice s takes list entries s, s + r, ... of every tile and the
//    slices are summed through LDS at the end;
//  * the list is walked in tiles of 64 entries: each lane gathers one entry
//    by index (particle by slot, superparticle by cell id -- the same
//    {x, y, z, m} FP64 record), converts it to FP32 offsets and stores it in
//    LDS; every lane then reads the tile back as broadcasts;
//  * FP32 arithmetic with per-tile partial sums added into the totals;
//    the potential of the particle on itself is removed at the end;
//  * workgroup ids are remapped so that each XCD (workgroups are dealt out
//    round-robin over the 8 XCDs) walks a contiguous stretch of groups,
//    which share most of their list entries in that XCD's L2.
// No MFMA: the pairwise sum is not a dense contraction.
#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kTile = 64;

__device__ __forceinline__ void mono(const float4 j, float xi, float yi,
                                     float zi, float eps2, float& ax,
                                     float& ay, float& az, float& ph) {
  const float dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float mr = j.w * rinv;
  const float mr3 = mr * rinv * rinv;
  ax = fmaf(mr3, dx, ax);
  ay = fmaf(mr3, dy, ay);
  az = fmaf(mr3, dz, az);
  ph -= mr;
}

// Second-order expansion of the softened kernel about the centre of mass X:
// with d = X - x_i, f = (|d|^2 + eps^2)^-1/2, S the second moments, q =
// d.S.d and t = tr S:
//   phi = -M f - (3 q f^2 - t) f^3 / 2
//   a   = d (M f^3 + 15/2 q f^7 - 3/2 t f^5) - 3 f^5 S d
__device__ __forceinline__ void quadr(const float4 j, const float4 qa,
                                      const float4 qb, float xi, float yi,
                                      float zi, float eps2, float& ax,
                                      float& ay, float& az, float& ph) {
  const float dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
  const float f = __builtin_amdgcn_rsqf(r2);
  const float f2 = f * f;
  const float f3 = f2 * f;
  const float f5 = f3 * f2;
  const float f7 = f5 * f2;
  // qa = (xx, yy, zz, xy), qb = (xz, yz, tr, 0)
  const float sx = fmaf(qa.x, dx, fmaf(qa.w, dy, qb.x * dz));
  const float sy = fmaf(qa.w, dx, fmaf(qa.y, dy, qb.y * dz));
  const float sz = fmaf(qb.x, dx, fmaf(qb.y, dy, qa.z * dz));
  const float q = fmaf(dx, sx, fmaf(dy, sy, dz * sz));
  const float t = qb.z;
  const float coef = fmaf(j.w, f3, fmaf(7.5f * q, f7, -1.5f * t * f5));
  const float f53 = 3.0f * f5;
  ax = fmaf(coef, dx, fmaf(-f53, sx, ax));
  ay = fmaf(coef, dy, fmaf(-f53, sy, ay));
  az = fmaf(coef, dz, fmaf(-f53, sz, az));
  ph -= fmaf(j.w, f, 0.5f * fmaf(3.0f * q, f2, -t) * f3);
}

template <int ORDER>
__global__ void __launch_bounds__(64)
k_force(const uint4* __restrict__ wi, int64_t n_wi, int64_t per_xcd,
        const uint32_t* __restrict__ g_cell, const double4* __restrict__ geo,
        const uint64_t* __restrict__ epj_off,
        const uint32_t* __restrict__ epj,
        const uint64_t* __restrict__ spj_off,
        const uint32_t* __restrict__ spj, const double4* __restrict__ pos,
        const double4* __restrict__ pm, const float4* __restrict__ quad,
        float eps2, float G, float4* __restrict__ acc) {
  __shared__ float4 tile[kTile];
  __shared__ float4 tq[ORDER == 2 ? 2 * kTile : 1];
  __shared__ float4 red[kTile];

  const uint32_t bid = blockIdx.x;
  const int64_t w = (int64_t)(bid & 7u) * per_xcd + (int64_t)(bid >> 3);
  if (w >= n_wi) return;  // uniform over the workgroup
  const uint4 it = wi[w];
  const int lane = threadIdx.x;
  const int ni = (int)it.z;          // 1..64
  const int r = kTile / ni;          // lane slices
  const int sl = lane / ni;
  const int ii = lane - sl * ni;
  const bool act = sl < r;
  const uint32_t g = it.x;
  const double4 cg = geo[g_cell[g]];

  float xi = 0.f, yi = 0.f, zi = 0.f, mi = 0.f;
  if (act) {
    const double4 p = pos[it.y + ii];
    xi = (float)(p.x - cg.x);
    yi = (float)(p.y - cg.y);
    zi = (float)(p.z - cg.z);
    mi = (float)p.w;
  }
  const uint64_t e0 = epj_off[g], ne = epj_off[g + 1] - e0;
  const uint64_t s0 = spj_off[g], ns = spj_off[g + 1] - s0;
  const uint64_t nl = ORDER == 1 ? ne + ns : ne;

  float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
  for (uint64_t tb = 0; tb < nl; tb += kTile) {
    const uint64_t q = tb + lane;
    float4 jd = make_float4(0.f, 0.f, 0.f, 0.f);  // massless padding
    if (q < nl) {
      double4 P;
      if (q < ne)
        P = pos[epj[e0 + q]];
      else
        P = pm[spj[s0 + (q - ne)]];
      jd = make_float4((float)(P.x - cg.x), (float)(P.y - cg.y),
                       (float)(P.z - cg.z), (float)P.w);
    }
    __syncthreads();
    tile[lane] = jd;
    __syncthreads();
    if (act) {
      float tx = 0.f, ty = 0.f, tz = 0.f, tp = 0.f;
      if (r == 1) {
#pragma unroll 8
        for (int k = 0; k < kTile; ++k)
          mono(tile[k], xi, yi, zi, eps2, tx, ty, tz, tp);
      } else {
        for (int k = sl; k < kTile; k += r)
          mono(tile[k], xi, yi, zi, eps2, tx, ty, tz, tp);
      }
      ax += tx;
      ay += ty;
      az += tz;
      ph += tp;
    }
  }
  if (ORDER == 2) {
    for (uint64_t tb = 0; tb < ns; tb += kTile) {
      const uint64_t q = tb + lane;
      float4 jd = make_float4(0.f, 0.f, 0.f, 0.f);
      float4 qa = make_float4(0.f, 0.f, 0.f, 0.f);
      float4 qb = make_float4(0.f, 0.f, 0.f, 0.f);
      if (q < ns) {
        const uint32_t cc = spj[s0 + q];
        const double4 P = pm[cc];
        jd = make_float4((float)(P.x - cg.x), (float)(P.y - cg.y),
                         (float)(P.z - cg.z), (float)P.w);
        qa = quad[2 * (int64_t)cc];
        qb = quad[2 * (int64_t)cc + 1];
        qb.z = qa.x + qa.y + qa.z;
      }
      __syncthreads();
      tile[lane] = jd;
      tq[2 * lane] = qa;
      tq[2 * lane + 1] = qb;
      __syncthreads();
      if (act) {
        float tx = 0.f, ty = 0.f, tz = 0.f, tp = 0.f;
        for (int k = sl; k < kTile; k += r)
          quadr(tile[k], tq[2 * k], tq[2 * k + 1], xi, yi, zi, eps2, tx, ty,
                tz, tp);
        ax += tx;
        ay += ty;
        az += tz;
        ph += tp;
      }
    }
  }
  if (r > 1) {
    __syncthreads();
    red[lane] = make_float4(ax, ay, az, ph);
    __syncthreads();
    if (lane < ni) {
      ax = ay = az = ph = 0.f;
      for (int s = 0; s < r; ++s) {
        const float4 v = red[s * ni + lane];
        ax += v.x;
        ay += v.y;
        az += v.z;
        ph += v.w;
      }
    }
  }
  if (lane < ni) {
    // the list holds the particle itself: it added exactly m_i / eps to
    // the potential (zero to the acceleration); take it out again
    ph += mi * __builtin_amdgcn_rsqf(eps2);
    acc[it.y + lane] = make_float4(G * ax, G * ay, G * az, G * ph);
  }
}

}  // namespace

int launch_force(nb_ctx* c) {
  int rc = reserve(c, c->acc, (size_t)c->n);
  if (rc) return rc;
  if (c->n_wi <= 0) return NB_OK;
  const int64_t per_xcd = (c->n_wi + 7) / 8;
  const int64_t nblk = per_xcd * 8;
  if (nblk > 0x7FFFFFFFLL)
    return set_err(c, NB_ERR_INPUT, "too many force work items");
  const float eps2 = (float)(c->cfg.eps * c->cfg.eps);
  const float G = (float)c->cfg.G;
  auto k = c->cfg.order == 2 ? k_force<2> : k_force<1>;
  hipLaunchKernelGGL(k, dim3((unsigned)nblk), dim3(kTile), 0, c->stream,
                     (const uint4*)c->wi.p, c->n_wi, per_xcd,
                     (const uint32_t*)c->g_cell.p, (const double4*)c->c_geo.p,
                     (const uint64_t*)c->epj_off.p, (const uint32_t*)c->epj.p,
                     (const uint64_t*)c->spj_off.p, (const uint32_t*)c->spj.p,
                     (const double4*)c->pos.p, (const double4*)c->c_pm.p,
                     (const float4*)c->c_quad.p, eps2, G, c->acc.p);
  return hip_check(c, hipGetLastError(), "force launch");
}

}  // namespace nb
