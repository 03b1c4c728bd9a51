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
//    slices; each slice sums its own block of every tile and the slices are
//    added through LDS at the end;
//  * the list is walked in tiles of 64 min(r, 4) entries: each lane gathers
//    entries by index (particle by slot, superparticle by cell id -- the
//    same {x, y, z, m} FP64 record), converts them to FP32 offsets and
//    stores them in LDS; the lanes of a slice then read its block back as
//    broadcasts;
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

// Sum of one slice's block of `cnt` tile entries (cnt <= 64).  Full blocks
// take the unrolled path; LDS offsets are then immediates.
template <int ORDER>
__device__ __forceinline__ void slice_sum(const float4* __restrict__ t,
                                          const float4* __restrict__ q,
                                          int cnt, float xi, float yi,
                                          float zi, float eps2, float& ax,
                                          float& ay, float& az, float& ph) {
  float tx = 0.f, ty = 0.f, tz = 0.f, tp = 0.f;
  if (ORDER == 1) {
    if (cnt == kTile) {
#pragma unroll 8
      for (int k = 0; k < kTile; ++k)
        mono(t[k], xi, yi, zi, eps2, tx, ty, tz, tp);
    } else {
#pragma unroll 4
      for (int k = 0; k < cnt; ++k)
        mono(t[k], xi, yi, zi, eps2, tx, ty, tz, tp);
    }
  } else {
    for (int k = 0; k < cnt; ++k)
      quadr(t[k], q[2 * k], q[2 * k + 1], xi, yi, zi, eps2, tx, ty, tz, tp);
  }
  ax += tx;
  ay += ty;
  az += tz;
  ph += tp;
}

constexpr int kMaxSlices = 4;
constexpr int kBigTile = kTile * kMaxSlices;

// One group chunk per wavefront.  With r = 64 / n_i lane slices (r <= 4),
// a tile holds 64 r list entries and slice s sums entries [64 s, 64 s + 64):
// every slice does the same unrolled work per tile as a full group does.
// For r > 4 the 256-entry tile is cut into r near-equal blocks.
struct ForceArgs {
  const uint32_t* __restrict__ g_cell;
  const CellRec* __restrict__ rec;
  const uint64_t* __restrict__ epj_off;
  const uint32_t* __restrict__ epj;
  const uint64_t* __restrict__ spj_off;
  const uint32_t* __restrict__ spj;
  const double4* __restrict__ pos;
  const double4* __restrict__ pm;
  const float4* __restrict__ quad;
  float eps2, G;
  float4* __restrict__ acc;
};

// The forces on one work item (wi = {group, first particle, count}); all 64
// lanes of the workgroup call it.
template <int ORDER>
__device__ __forceinline__ void force_item(const uint4 it, const ForceArgs& A,
                                           float4* tile, float4* tq,
                                           float4* red) {
  const uint32_t* __restrict__ g_cell = A.g_cell;
  const CellRec* __restrict__ rec = A.rec;
  const uint64_t* __restrict__ epj_off = A.epj_off;
  const uint32_t* __restrict__ epj = A.epj;
  const uint64_t* __restrict__ spj_off = A.spj_off;
  const uint32_t* __restrict__ spj = A.spj;
  const double4* __restrict__ pos = A.pos;
  const double4* __restrict__ pm = A.pm;
  const float4* __restrict__ quad = A.quad;
  const float eps2 = A.eps2, G = A.G;
  float4* __restrict__ acc = A.acc;
  const int lane = threadIdx.x;
  const int ni = (int)it.z;            // 1..64
  const int r = kTile / ni;            // lane slices
  const int sl = lane / ni;
  const int ii = lane - sl * ni;
  const bool act = sl < r;
  const int q = r < kMaxSlices ? r : kMaxSlices;  // tile = 64 q entries
  const int T = kTile * q;
  // this slice's block of a full tile
  const int blk0 = r <= kMaxSlices ? sl * kTile : (sl * T) / r;
  const int blk1 = r <= kMaxSlices ? blk0 + kTile : ((sl + 1) * T) / r;
  const uint32_t g = it.x;
  const double4 cg = rec[g_cell[g]].geo;

  float xi = 0.f, yi = 0.f, zi = 0.f, mi = 0.f;
  if (act) {
    const double4 p = pos[it.y + ii];
    xi = (float)(p.x - cg.x);
    yi = (float)(p.y - cg.y);
    zi = (float)(p.z - cg.z);
    mi = (float)p.w;
  }
  // list entries are addressed relative to the group's list: [0, ne) are
  // particles, [ne, ne + ns) superparticles
  const uint64_t e0 = epj_off[g];
  const uint32_t ne = (uint32_t)(epj_off[g + 1] - e0);
  const uint64_t s0 = spj_off[g];
  const uint32_t ns = (uint32_t)(spj_off[g + 1] - s0);
  const uint32_t* __restrict__ ida = epj + e0;
  const uint32_t* __restrict__ idb = spj + s0;
  const uint32_t nl = ORDER == 1 ? ne + ns : ne;

  // ids of the tile starting at tb (slot u of this lane), kNone past the end
  auto load_ids = [&](uint32_t tb, uint32_t* id) {
#pragma unroll
    for (int u = 0; u < kMaxSlices; ++u) {
      id[u] = kNone;
      const uint32_t e = tb + (uint32_t)(u * kTile + lane);
      if (u < q && e < nl) id[u] = e < ne ? ida[e] : idb[e - ne];
    }
  };

  float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
  uint32_t nid[kMaxSlices];
  load_ids(0, nid);
  for (uint32_t tb = 0; tb < nl; tb += (uint32_t)T) {
    uint32_t cid[kMaxSlices];
    double4 P[kMaxSlices];
#pragma unroll
    for (int u = 0; u < kMaxSlices; ++u) {
      cid[u] = nid[u];
      const uint32_t e = tb + (uint32_t)(u * kTile + lane);
      if (cid[u] != kNone) P[u] = e < ne ? pos[cid[u]] : pm[cid[u]];
    }
    // the next tile's ids arrive while this tile is staged and summed
    if (tb + (uint32_t)T < nl) load_ids(tb + (uint32_t)T, nid);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMaxSlices; ++u) {
      if (u < q) {
        float4 jd = make_float4(0.f, 0.f, 0.f, 0.f);  // massless padding
        if (cid[u] != kNone)
          jd = make_float4((float)(P[u].x - cg.x), (float)(P[u].y - cg.y),
                           (float)(P[u].z - cg.z), (float)P[u].w);
        tile[u * kTile + lane] = jd;
      }
    }
    __syncthreads();
    if (act) {
      const int valid = nl - tb < (uint32_t)T ? (int)(nl - tb) : T;
      const int hi = blk1 < valid ? blk1 : valid;
      const int cnt = hi > blk0 ? hi - blk0 : 0;
      slice_sum<1>(tile + blk0, nullptr, cnt, xi, yi, zi, eps2, ax, ay, az,
                   ph);
    }
  }
  if (ORDER == 2) {
    for (uint32_t tb = 0; tb < ns; tb += (uint32_t)T) {
      uint32_t cid[kMaxSlices];
#pragma unroll
      for (int u = 0; u < kMaxSlices; ++u) {
        const uint32_t e = tb + (uint32_t)(u * kTile + lane);
        cid[u] = (u < q && e < ns) ? idb[e] : kNone;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kMaxSlices; ++u) {
        if (u < q) {
          float4 jd = make_float4(0.f, 0.f, 0.f, 0.f);
          float4 qa = make_float4(0.f, 0.f, 0.f, 0.f);
          float4 qb = make_float4(0.f, 0.f, 0.f, 0.f);
          if (cid[u] != kNone) {
            const double4 Q = pm[cid[u]];
            jd = make_float4((float)(Q.x - cg.x), (float)(Q.y - cg.y),
                             (float)(Q.z - cg.z), (float)Q.w);
            qa = quad[2 * (int64_t)cid[u]];
            qb = quad[2 * (int64_t)cid[u] + 1];
            qb.z = qa.x + qa.y + qa.z;
          }
          const int slot = u * kTile + lane;
          tile[slot] = jd;
          tq[2 * slot] = qa;
          tq[2 * slot + 1] = qb;
        }
      }
      __syncthreads();
      if (act) {
        const int valid = ns - tb < (uint32_t)T ? (int)(ns - tb) : T;
        const int hi = blk1 < valid ? blk1 : valid;
        const int cnt = hi > blk0 ? hi - blk0 : 0;
        slice_sum<2>(tile + blk0, tq + 2 * blk0, cnt, xi, yi, zi, eps2, ax,
                     ay, az, ph);
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

// One launch, one workgroup (one wavefront) per work item; workgroup ids are
// remapped so each XCD takes a contiguous stretch of work items.
template <int ORDER>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_force(const uint4* __restrict__ wi, int64_t n_wi, int64_t per_xcd,
        ForceArgs A) {
  __shared__ float4 tile[kBigTile];
  __shared__ float4 tq[ORDER == 2 ? 2 * kBigTile : 1];
  __shared__ float4 red[kTile];
  const uint32_t bid = blockIdx.x;
  const int64_t w = (int64_t)(bid & 7u) * per_xcd + (int64_t)(bid >> 3);
  if (w >= n_wi) return;  // uniform over the workgroup
  force_item<ORDER>(wi[w], A, tile, tq, red);
}

// Persistent form: a fixed number of resident workgroups, each pulling the
// next work item of its XCD's contiguous stretch from that XCD's counter
// (queue[0..7], zeroed before the launch) until the stretch is used up.
template <int ORDER>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_force_queue(const uint4* __restrict__ wi, int64_t n_wi, int64_t per_xcd,
              unsigned int* __restrict__ queue, ForceArgs A) {
  __shared__ float4 tile[kBigTile];
  __shared__ float4 tq[ORDER == 2 ? 2 * kBigTile : 1];
  __shared__ float4 red[kTile];
  const uint32_t x = blockIdx.x & 7u;
  const int64_t lo = (int64_t)x * per_xcd;
  const int64_t hi = lo + per_xcd < n_wi ? lo + per_xcd : n_wi;
  for (;;) {
    unsigned int k = 0;
    if (threadIdx.x == 0) k = atomicAdd(&queue[x], 1u);
    k = __shfl(k, 0, 64);
    const int64_t w = lo + (int64_t)k;
    if (w >= hi) break;  // uniform over the workgroup
    force_item<ORDER>(wi[w], A, tile, tq, red);
    __syncthreads();  // the next item reuses the tile and reduction space
  }
}

__global__ void k_zero_queue(unsigned int* q) {
  if (threadIdx.x < 8) q[threadIdx.x] = 0u;
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
  ForceArgs A;
  A.g_cell = c->g_cell.p;
  A.rec = c->c_rec.p;
  A.epj_off = c->epj_off.p;
  A.epj = c->epj.p;
  A.spj_off = c->spj_off.p;
  A.spj = c->spj.p;
  A.pos = c->pos.p;
  A.pm = c->c_pm.p;
  A.quad = c->c_quad.p;
  A.eps2 = (float)(c->cfg.eps * c->cfg.eps);
  A.G = (float)c->cfg.G;
  A.acc = c->acc.p;
  if (c->cfg.flags & NB_FLAG_PERSISTENT) {
    if ((rc = reserve(c, c->queue, 8))) return rc;
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, c->stream,
                       c->queue.p);
    // resident workgroups: 256 CUs x 16 one-wave workgroups (4 per SIMD,
    // the kernel's occupancy), dealt round-robin over the 8 XCDs
    int64_t nq = 256 * 16;
    if (nq > nblk) nq = nblk;
    nq = (nq + 7) / 8 * 8;
    auto k = c->cfg.order == 2 ? k_force_queue<2> : k_force_queue<1>;
    hipLaunchKernelGGL(k, dim3((unsigned)nq), dim3(kTile), 0, c->stream,
                       (const uint4*)c->wi.p, c->n_wi, per_xcd, c->queue.p, A);
  } else {
    auto k = c->cfg.order == 2 ? k_force<2> : k_force<1>;
    hipLaunchKernelGGL(k, dim3((unsigned)nblk), dim3(kTile), 0, c->stream,
                       (const uint4*)c->wi.p, c->n_wi, per_xcd, A);
  }
  return hip_check(c, hipGetLastError(), "force launch");
}

}  // namespace nb
