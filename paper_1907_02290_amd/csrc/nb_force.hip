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
//  * the list is walked in tiles of 64 min(r, KMAX) entries (KMAX 3 for
//    the monopole and 2 for the quadrupole kernel by default), first its
//    particles (by slot), then its superparticles (by cell id; the same
//    {x, y, z, m} FP64 record): each lane gathers entries by index, converts
//    them to FP32 offsets and stores them in LDS; the lanes of a slice then
//    read its block back as broadcasts, each block shifted by one pad entry
//    so that the slices' simultaneous reads fall on different LDS banks;
//  * FP32 arithmetic with per-tile partial sums added into the totals;
//    the potential of the particle on itself is removed at the end;
//  * workgroup ids are remapped so that each XCD (workgroups are dealt out
//    round-robin over the 8 XCDs) walks a contiguous stretch of groups,
//    which share most of their list entries in that XCD's L2.
// No MFMA: the pairwise sum is not a dense contraction.
#include <algorithm>

#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kTile = 64;

// One monopole term; the first term of a block assigns the partial sums
// instead of adding to them (no zero initialisation).
template <bool FIRST>
__device__ __forceinline__ void mono(const float4 j, float xi, float yi,
                                     float zi, float eps2, float& ax,
                                     float& ay, float& az, float& ph) {
  const float dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
  const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float mr = j.w * rinv;
  const float mr3 = mr * rinv * rinv;
  if (FIRST) {
    ax = mr3 * dx;
    ay = mr3 * dy;
    az = mr3 * dz;
    ph = -mr;
  } else {
    ax = fmaf(mr3, dx, ax);
    ay = fmaf(mr3, dy, ay);
    az = fmaf(mr3, dz, az);
    ph -= mr;
  }
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

// Adds the sum over one slice's block of `cnt` staged entries (cnt <= 64)
// to the totals; the block's partial sums are kept apart and added once.
// A full block is unrolled completely, so its LDS offsets are immediates.
template <int ORDER>
__device__ __forceinline__ void slice_sum(const float4* __restrict__ t,
                                          const float4* __restrict__ q,
                                          int cnt, float xi, float yi,
                                          float zi, float eps2, float& ax,
                                          float& ay, float& az, float& ph) {
  if (cnt <= 0) return;
  float tx, ty, tz, tp;
  if (ORDER == 1) {
    mono<true>(t[0], xi, yi, zi, eps2, tx, ty, tz, tp);
    if (cnt == kTile) {
#pragma unroll
      for (int k = 1; k < kTile; ++k)
        mono<false>(t[k], xi, yi, zi, eps2, tx, ty, tz, tp);
    } else {
#pragma unroll 4
      for (int k = 1; k < cnt; ++k)
        mono<false>(t[k], xi, yi, zi, eps2, tx, ty, tz, tp);
    }
  } else {
    tx = ty = tz = tp = 0.f;
    for (int k = 0; k < cnt; ++k)
      quadr(t[k], q[2 * k], q[2 * k + 1], xi, yi, zi, eps2, tx, ty, tz, tp);
  }
  ax += tx;
  ay += ty;
  az += tz;
  ph += tp;
}

// Largest tile, in 64-entry blocks (KMAX): by default 3 for the monopole
// kernel, whose prefetched records (one FP64 record per slice and lane) then
// fit six waves per SIMD (79 VGPRs; with 4 blocks it needed 93, five
// waves), and 2 for the quadrupole kernel, which stages 2 x 16 bytes of
// second moments per entry besides the record, so that its LDS (and so its
// occupancy) stays in line with its registers.  The configuration can pick
// 1 to 4 blocks (nb_config.tile_j = 64 KMAX entries) and the occupancy the
// register allocation aims at (nb_config.waves_per_simd: 4, 6 or 8); the
// autotuner chooses among these instances.
constexpr int kDefaultSlices[3] = {0, 3, 2};
constexpr int kDefaultWaves = 6;

template <int ORDER, int KMAX>
struct Tiles {
  static constexpr int kMaxSlices = KMAX;
  static constexpr int kBig = kTile * KMAX;
  // LDS entries of a tile: one pad entry after each slice's block, for up
  // to kPad blocks (the slices past that share the last shift).  The
  // quadrupole kernel stages 48 bytes per entry, and 64 pads would cost it
  // a quarter of its occupancy; its slices past 16 (chunks of three
  // particles or fewer) share one shift.
  static constexpr int kPad = ORDER == 2 ? 16 : kTile;
  static constexpr int kLds = kBig + kPad;
};

// One group chunk per wavefront.  With r = 64 / n_i lane slices (r up to
// the kernel's largest slice count, kMaxSlices), a tile holds 64 r list
// entries and slice s sums entries [64 s, 64 s + 64): every slice does the
// same unrolled work per tile as a full group does.  For larger r the
// largest tile is cut into r near-equal blocks.  The slices' sums are added
// through LDS at the end, in the tile's space.
// Lists: group g's particle ids start at epj[epj_off[g]] and number
// cnt_e[g], its superparticle ids at spj[spj_off[g]], cnt_s[g] of them (the
// offsets are where the lists start; in refresh mode each group's list has
// room to grow past its length).
struct ForceArgs {
  const uint32_t* __restrict__ g_cell;
  const CellRec* __restrict__ rec;
  const uint64_t* __restrict__ epj_off;
  const uint32_t* __restrict__ epj;
  const uint64_t* __restrict__ spj_off;
  const uint32_t* __restrict__ spj;
  const uint32_t* __restrict__ cnt_e;
  const uint32_t* __restrict__ cnt_s;
  const double4* __restrict__ pos;
  const double4* __restrict__ pm;
  const float4* __restrict__ quad;
  const float4* __restrict__ jcopy;  // copied lists (COPIED), else unused
  float eps2, G;
  float4* __restrict__ acc;
};

// LDS position of entry e = 64 u + lane of a tile (see force_item): e plus
// one pad entry per block before its own, where its block is u when the
// blocks are the tile's 64-entry thirds, quarters... (r <= KMAX), else
// (r (e + 1) - 1) / (64 KMAX) of r equal blocks; blocks past PAD - 1 share
// the shift of block PAD - 1.
template <int KMAX, int PAD>
__device__ __forceinline__ int tile_pos(int e, int u, int r) {
  int b = r <= KMAX ? u : (r * (e + 1) - 1) / (kTile * KMAX);
  if constexpr (PAD < kTile) b = b < PAD - 1 ? b : PAD - 1;
  return e + b;
}

// One slice's share of a tile of T entries of which `valid` are filled.
__device__ __forceinline__ int block_count(int valid, int blk0, int blk1) {
  const int hi = blk1 < valid ? blk1 : valid;
  return hi - blk0;
}

// The forces on one work item (wi = {group, first particle, count}); all 64
// lanes of the workgroup call it.  The list is taken in two segments, its
// particles (ids into the particle array) and its superparticles (ids into
// the cell array), so every tile reads from one array.  Entries past the end
// of a segment are staged as duplicates of its last entry and never summed.
// COPIED (monopole only): the group's entries were copied beforehand, as
// FP32 offsets from its centre, to jcopy[epj_off + spj_off ...] (k_copy_j),
// and the tiles are read from there.
template <int ORDER, bool COPIED, int KMAX>
__device__ __forceinline__ void force_item(const uint4 it, const ForceArgs& A,
                                           float4* tile, float4* tq,
                                           float4* red) {
  const uint32_t* __restrict__ g_cell = A.g_cell;
  const CellRec* __restrict__ rec = A.rec;
  const float4* __restrict__ quad = A.quad;
  const float eps2 = A.eps2, G = A.G;
  float4* __restrict__ acc = A.acc;
  const int lane = threadIdx.x;
  const int ni = (int)it.z;            // 1..64
  const int r = kTile / ni;            // lane slices
  const int sl = lane / ni;
  const int ii = lane - sl * ni;
  const bool act = sl < r;
  constexpr int kMaxSlices = Tiles<ORDER, KMAX>::kMaxSlices;
  constexpr int kPad = Tiles<ORDER, KMAX>::kPad;
  const int q = r < kMaxSlices ? r : kMaxSlices;  // tile = 64 q entries
  const int T = kTile * q;
  // this slice's block of a full tile
  const int blk0 = r <= kMaxSlices ? sl * kTile : (sl * T) / r;
  const int blk1 = r <= kMaxSlices ? blk0 + kTile : ((sl + 1) * T) / r;
  // In LDS each block is followed by one pad entry, so that block s starts
  // at blk0 + s: the slices of a wave read their blocks at the same time,
  // and blocks 64 entries apart would otherwise sit on the same LDS banks
  // (16-byte entries; one pad shifts the next block by four banks).  Entry
  // e of a tile, in block (r (e + 1) - 1) / T, goes to e + that block, or
  // e + kPad - 1 past kPad - 1 blocks.
  const int tbase = blk0 + (kPad < kTile && sl > kPad - 1 ? kPad - 1 : sl);
  const uint32_t g = it.x;
  const double4 cg = rec[g_cell[g]].geo;

  float xi = 0.f, yi = 0.f, zi = 0.f, mi = 0.f;
  if (act) {
    const double4 p = A.pos[it.y + ii];
    xi = (float)(p.x - cg.x);
    yi = (float)(p.y - cg.y);
    zi = (float)(p.z - cg.z);
    mi = (float)p.w;
  }
  const uint64_t e0 = A.epj_off[g];
  const uint32_t ne = A.cnt_e[g];
  const uint64_t s0 = A.spj_off[g];
  const uint32_t ns = A.cnt_s[g];

  float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
  // monopole: both segments; quadrupole: the particle segment here, the
  // superparticles with their second moments below
  for (int seg = 0; seg < (ORDER == 1 ? 2 : 1); ++seg) {
    if (COPIED) {
      const uint32_t n = seg ? ns : ne;
      if (n == 0) continue;
      const uint32_t last = n - 1;
      const float4* __restrict__ jc = A.jcopy + (e0 + s0) + (seg ? ne : 0u);
      float4 J[kMaxSlices];
#pragma unroll
      for (int u = 0; u < kMaxSlices; ++u) {
        if (u < q) {
          const uint32_t e = (uint32_t)(u * kTile + lane);
          J[u] = jc[e < last ? e : last];
        }
      }
      for (uint32_t tb = 0; tb < n; tb += (uint32_t)T) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kMaxSlices; ++u)
          if (u < q) tile[tile_pos<KMAX, kPad>(u * kTile + lane, u, r)] = J[u];
        const uint32_t nb = tb + (uint32_t)T;
        if (nb < n) {
#pragma unroll
          for (int u = 0; u < kMaxSlices; ++u) {
            if (u < q) {
              const uint32_t e = nb + (uint32_t)(u * kTile + lane);
              J[u] = jc[e < last ? e : last];
            }
          }
        }
        __syncthreads();
        if (act) {
          const int valid = n - tb < (uint32_t)T ? (int)(n - tb) : T;
          slice_sum<1>(tile + tbase, nullptr, block_count(valid, blk0, blk1),
                       xi, yi, zi, eps2, ax, ay, az, ph);
        }
      }
      continue;
    }
    const uint32_t* __restrict__ ids = seg ? A.spj + s0 : A.epj + e0;
    const double4* __restrict__ src = seg ? A.pm : A.pos;
    const uint32_t n = seg ? ns : ne;
    if (n == 0) continue;
    const uint32_t last = n - 1;
    uint32_t nid[kMaxSlices];
    double4 P[kMaxSlices];
    // records of the first tile, ids of the second
#pragma unroll
    for (int u = 0; u < kMaxSlices; ++u) {
      if (u < q) {
        const uint32_t e = (uint32_t)(u * kTile + lane);
        P[u] = src[ids[e < last ? e : last]];
        const uint32_t e2 = (uint32_t)T + e;
        nid[u] = ids[e2 < last ? e2 : last];
      }
    }
    for (uint32_t tb = 0; tb < n; tb += (uint32_t)T) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kMaxSlices; ++u)
        if (u < q)
          tile[tile_pos<KMAX, kPad>(u * kTile + lane, u, r)] = make_float4(
              (float)(P[u].x - cg.x), (float)(P[u].y - cg.y),
              (float)(P[u].z - cg.z), (float)P[u].w);
      // the next tile's records and the ids of the one after arrive while
      // this tile is summed
      const uint32_t nb = tb + (uint32_t)T;
      if (nb < n) {
#pragma unroll
        for (int u = 0; u < kMaxSlices; ++u) {
          if (u < q) {
            P[u] = src[nid[u]];
            const uint32_t e = nb + (uint32_t)T + (uint32_t)(u * kTile + lane);
            nid[u] = ids[e < last ? e : last];
          }
        }
      }
      __syncthreads();
      if (act) {
        const int valid = n - tb < (uint32_t)T ? (int)(n - tb) : T;
        slice_sum<1>(tile + tbase, nullptr, block_count(valid, blk0, blk1),
                     xi, yi, zi, eps2, ax, ay, az, ph);
      }
    }
  }
  if (ORDER == 2 && ns > 0) {
    const uint32_t* __restrict__ ids = A.spj + s0;
    const uint32_t last = ns - 1;
    for (uint32_t tb = 0; tb < ns; tb += (uint32_t)T) {
      uint32_t cid[kMaxSlices];
#pragma unroll
      for (int u = 0; u < kMaxSlices; ++u) {
        if (u < q) {
          const uint32_t e = tb + (uint32_t)(u * kTile + lane);
          cid[u] = ids[e < last ? e : last];
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kMaxSlices; ++u) {
        if (u < q) {
          const double4 Q = A.pm[cid[u]];
          float4 qa = quad[2 * (int64_t)cid[u]];
          float4 qb = quad[2 * (int64_t)cid[u] + 1];
          qb.z = qa.x + qa.y + qa.z;
          const int slot = tile_pos<KMAX, kPad>(u * kTile + lane, u, r);
          tile[slot] = make_float4((float)(Q.x - cg.x), (float)(Q.y - cg.y),
                                   (float)(Q.z - cg.z), (float)Q.w);
          tq[2 * slot] = qa;
          tq[2 * slot + 1] = qb;
        }
      }
      __syncthreads();
      if (act) {
        const int valid = ns - tb < (uint32_t)T ? (int)(ns - tb) : T;
        slice_sum<2>(tile + tbase, tq + 2 * tbase,
                     block_count(valid, blk0, blk1), xi, yi, zi, eps2, ax,
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

// Launch plan: XCD x takes the work items [b[x], b[x + 1]), a contiguous
// stretch (its groups' tree neighbourhoods share that XCD's L2), and the
// stretches are cut where the estimated cost is balanced.  Workgroups are
// dealt to the XCDs round-robin, so workgroup bid runs item
// b[bid & 7] + (bid >> 3).
// The last kTailItems items of each stretch (the launch's tail) are taken
// longest first: item tail[x kTailItems + k] for position ws[x] + k (order
// NULL, or ws[x] = b[x + 1]: no reordering).  Only the tail leaves Morton
// order, so the L2 sharing between neighbouring groups is kept for the rest.
constexpr int kTailItems = 2048;

struct XcdPlan {
  int64_t b[9];
  int64_t ws[8];
  const uint32_t* tail;
};

__device__ __forceinline__ int64_t plan_item(const XcdPlan& plan, uint32_t x,
                                             int64_t j) {
  return (plan.tail && j >= plan.ws[x])
             ? (int64_t)plan.tail[x * kTailItems + (j - plan.ws[x])]
             : j;
}

// The tail order t in the plan, when it was made for the same stretches.
void use_tail(const TailOrder& t, XcdPlan& plan) {
  if (!t.valid || !std::equal(t.b, t.b + 9, plan.b)) return;
  for (int x = 0; x < 8; ++x)
    plan.ws[x] = std::max(plan.b[x], plan.b[x + 1] - (int64_t)kTailItems);
  plan.tail = t.order.p;
}

// The plan b as a kernel argument; a plan that does not cover the n_wi
// items (none computed for them) is replaced by equal stretches.  Returns
// the grid size: 8 x the longest stretch.
int64_t checked_plan(int64_t n_wi, int64_t* b, XcdPlan& plan) {
  bool ok = b[0] == 0 && b[8] == n_wi;
  for (int x = 0; x < 8; ++x) ok = ok && b[x] <= b[x + 1];
  if (!ok) {
    const int64_t per = (n_wi + 7) / 8;
    for (int x = 0; x <= 8; ++x) b[x] = std::min<int64_t>(x * per, n_wi);
  }
  int64_t most = 0;
  for (int x = 0; x < 9; ++x) plan.b[x] = b[x];
  for (int x = 0; x < 8; ++x) {
    plan.ws[x] = b[x + 1];
    most = std::max(most, b[x + 1] - b[x]);
  }
  plan.tail = nullptr;
  return most * 8;
}

// One launch, one workgroup (one wavefront) per work item, with tiles of
// KMAX 64-entry blocks and registers allotted for WAVES waves per SIMD (the
// next tile's records are held in registers).
template <int ORDER, bool COPIED, int KMAX, int WAVES>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(WAVES, 8)))
k_force(const uint4* __restrict__ wi, XcdPlan plan, ForceArgs A) {
  __shared__ float4 tile[Tiles<ORDER, KMAX>::kLds];
  __shared__ float4 tq[ORDER == 2 ? 2 * Tiles<ORDER, KMAX>::kLds : 1];
  const uint32_t bid = blockIdx.x;
  const uint32_t x = bid & 7u;
  const int64_t j = plan.b[x] + (int64_t)(bid >> 3);
  if (j >= plan.b[x + 1]) return;  // uniform over the workgroup
  force_item<ORDER, COPIED, KMAX>(wi[plan_item(plan, x, j)], A, tile, tq,
                                  tile);
}

// Estimated cost of a group's work items, in list entries per lane slice:
// a chunk of n_i particles runs on r = 64 / n_i slices over tiles of 64 q
// entries (q = min(r, largest slice count)), every slice taking 64 q / r
// entries of each tile, for the particle and the superparticle segment
// separately; plus about one tile for loading the chunk and the final sums.
// Quadrupole superparticles count twice.
// KMAX: the kernel's largest slice count (tiles of 64 q entries,
// q = min(r, KMAX)); WS: weight of a superparticle entry.  The SPH density
// kernel takes tiles of 64 entries (KMAX 1) and has no superparticles.
template <int KMAX, int WS>
__device__ inline uint64_t item_cost(uint64_t ne, uint64_t ns, int ni) {
  const int r = kTile / ni;
  const int q = r < KMAX ? r : KMAX;
  const uint64_t T = (uint64_t)kTile * (uint64_t)q;
  const uint64_t tiles = (ne + T - 1) / T + (uint64_t)WS * ((ns + T - 1) / T);
  return tiles * T / (uint64_t)r + (uint64_t)kTile;
}

template <int KMAX, int WS>
__global__ void __launch_bounds__(256)
k_group_cost(int64_t n_groups, const uint32_t* __restrict__ g_chunks,
             const uint4* __restrict__ wi, const uint32_t* __restrict__ cnt_e,
             const uint32_t* __restrict__ cnt_s,
             uint32_t* __restrict__ cost) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const uint64_t ne = cnt_e[g];
  const uint64_t ns = cnt_s ? cnt_s[g] : 0u;
  uint64_t sum = 0;
  for (uint32_t w = g_chunks[g]; w < g_chunks[g + 1]; ++w)
    sum += item_cost<KMAX, WS>(ne, ns, (int)wi[w].z);
  cost[g] = sum < 0xFFFFFFFFull ? (uint32_t)sum : 0xFFFFFFFFu;
}

// The plan from the scanned group costs (off[n_groups] = total): the cut
// before XCD x is at the first group whose cost prefix reaches x / 8 of the
// total, turned into a work-item index by the groups' chunk offsets.
__global__ void k_xcd_split(int64_t n_groups, const uint64_t* __restrict__ off,
                            const uint32_t* __restrict__ g_chunks,
                            uint64_t* __restrict__ plan) {
  const int x = (int)threadIdx.x;
  if (x > 8) return;
  const uint64_t total = off[n_groups];
  int64_t g = x == 8 ? n_groups : 0;
  if (x > 0 && x < 8) {
    const uint64_t target = (total / 8) * (uint64_t)x +
                            ((total % 8) * (uint64_t)x) / 8;
    int64_t lo = 0, hi = n_groups;  // smallest g with off[g] >= target
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (off[mid] >= target)
        hi = mid;
      else
        lo = mid + 1;
    }
    g = lo;
  }
  plan[x] = g_chunks[g];
}

// The tail of XCD x's stretch (its last kTailItems items, fewer if the
// stretch is shorter) sorted by estimated cost, longest first, ties in item
// order: a bitonic sort in LDS by one workgroup per XCD.
template <int KMAX, int WS>
__global__ void __launch_bounds__(1024)
k_tail_order(const uint4* __restrict__ wi,
             const uint32_t* __restrict__ cnt_e,
             const uint32_t* __restrict__ cnt_s, XcdPlan plan,
             uint32_t* __restrict__ tail) {
  __shared__ uint64_t key[kTailItems];
  const uint32_t x = blockIdx.x;
  const int64_t s0 = plan.ws[x];
  const int n = (int)(plan.b[x + 1] - s0);
  for (int i = threadIdx.x; i < kTailItems; i += blockDim.x) {
    uint64_t k = ~0ull;
    if (i < n) {
      const uint4 it = wi[s0 + i];
      const uint32_t g = it.x;
      uint64_t c = item_cost<KMAX, WS>(cnt_e[g], cnt_s[g], (int)it.z);
      if (c > 0xFFFFFFFEull) c = 0xFFFFFFFEull;
      k = ((uint64_t)(0xFFFFFFFFu - (uint32_t)c) << 32) | (uint32_t)i;
    }
    key[i] = k;
  }
  __syncthreads();
  for (int size = 2; size <= kTailItems; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < kTailItems; i += blockDim.x) {
        const int jx = i ^ stride;
        if (jx > i) {
          const bool up = (i & size) == 0;
          const uint64_t a = key[i], b = key[jx];
          if ((a > b) == up) {
            key[i] = b;
            key[jx] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    tail[x * kTailItems + i] = (uint32_t)(s0 + (int64_t)(key[i] & 0xFFFFFFFFu));
}

// Copied lists (the paper's method G1, for comparison with index lists):
// one wave per group writes every entry of its list, particles then
// superparticles, as an FP32 offset from the group's centre and the mass,
// to jc[epj_off[g] + spj_off[g] ...].  Groups are dealt to XCDs in
// contiguous stretches as in the force kernel.
__global__ void __launch_bounds__(256)
k_copy_j(int64_t n_groups, int64_t nblk, const uint32_t* __restrict__ g_cell,
         const CellRec* __restrict__ rec,
         const uint64_t* __restrict__ epj_off,
         const uint32_t* __restrict__ epj,
         const uint64_t* __restrict__ spj_off,
         const uint32_t* __restrict__ spj, const double4* __restrict__ pos,
         const double4* __restrict__ pm, float4* __restrict__ jc) {
  const int64_t per = (nblk + 7) / 8;
  const int64_t blk = (int64_t)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  if (blk >= nblk) return;
  const int64_t g = blk * 4 + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  if (g >= n_groups) return;
  const double4 cg = rec[g_cell[g]].geo;
  const uint64_t e0 = epj_off[g], s0 = spj_off[g];
  const uint32_t ne = (uint32_t)(epj_off[g + 1] - e0);
  const uint32_t ns = (uint32_t)(spj_off[g + 1] - s0);
  float4* __restrict__ out = jc + (e0 + s0);
  for (uint32_t e = lane; e < ne + ns; e += 64u) {
    const double4 P = e < ne ? pos[epj[e0 + e]] : pm[spj[s0 + (e - ne)]];
    out[e] = make_float4((float)(P.x - cg.x), (float)(P.y - cg.y),
                         (float)(P.z - cg.z), (float)P.w);
  }
}

// Persistent form: a fixed number of resident workgroups, each pulling the
// next work item of its XCD's contiguous stretch from that XCD's counter
// (queue[0..7], zeroed before the launch) until the stretch is used up.
template <int ORDER>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_force_queue(const uint4* __restrict__ wi, XcdPlan plan,
              unsigned int* __restrict__ queue, ForceArgs A) {
  constexpr int K = kDefaultSlices[ORDER];
  __shared__ float4 tile[Tiles<ORDER, K>::kLds];
  __shared__ float4 tq[ORDER == 2 ? 2 * Tiles<ORDER, K>::kLds : 1];
  const uint32_t x = blockIdx.x & 7u;
  const int64_t lo = plan.b[x];
  const int64_t hi = plan.b[x + 1];
  for (;;) {
    unsigned int k = 0;
    if (threadIdx.x == 0) k = atomicAdd(&queue[x], 1u);
    k = __shfl(k, 0, 64);
    const int64_t j = lo + (int64_t)k;
    if (j >= hi) break;  // uniform over the workgroup
    force_item<ORDER, false, K>(wi[plan_item(plan, x, j)], A, tile, tq,
                                tile);
    __syncthreads();  // the next item reuses the tile and reduction space
  }
}

// SPH density on the short-range neighbour lists (section 2's short-range
// interaction): rho_i = norm * sum_j m_j w(|x_i - x_j| / h) over the list
// of i's group, w the cubic spline of compact support (1 - 6 q^2 + 6 q^3 up
// to q = 1/2, 2 (1 - q)^3 up to 1, 0 beyond), norm = 8 / (pi h^3).  The
// work items, lane slices, FP32 offsets from the group centre and LDS tiles
// are the force kernel's; a slice takes a block of every 64-entry tile.
__global__ void __launch_bounds__(64)
k_density(const uint4* __restrict__ wi, XcdPlan plan,
          const uint32_t* __restrict__ g_cell,
          const CellRec* __restrict__ rec,
          const uint64_t* __restrict__ nb_off,
          const uint32_t* __restrict__ nb_ids,
          const double4* __restrict__ pos, float h2inv, float norm,
          float* __restrict__ rho) {
  __shared__ float4 tile[kTile];
  __shared__ float red[kTile];
  const uint32_t bid = blockIdx.x;
  const uint32_t x = bid & 7u;
  const int64_t w = plan.b[x] + (int64_t)(bid >> 3);
  if (w >= plan.b[x + 1]) return;  // uniform over the workgroup
  const uint4 it = wi[w];
  const int lane = threadIdx.x;
  const int ni = (int)it.z;
  const int r = kTile / ni;
  const int sl = lane / ni;
  const int ii = lane - sl * ni;
  const bool act = sl < r;
  const int blk0 = (sl * kTile) / r, blk1 = ((sl + 1) * kTile) / r;
  const uint32_t g = it.x;
  const double4 cg = rec[g_cell[g]].geo;
  float xi = 0.f, yi = 0.f, zi = 0.f;
  if (act) {
    const double4 p = pos[it.y + ii];
    xi = (float)(p.x - cg.x);
    yi = (float)(p.y - cg.y);
    zi = (float)(p.z - cg.z);
  }
  const uint64_t o0 = nb_off[g];
  const uint32_t n = (uint32_t)(nb_off[g + 1] - o0);
  const uint32_t last = n ? n - 1 : 0;
  float sum = 0.f;
  // the next tile's record and the id of the one after are loaded while a
  // tile is summed (as in the force kernel)
  double4 P = make_double4(0.0, 0.0, 0.0, 0.0);
  uint32_t nid = 0;
  if (n > 0) {
    const uint32_t e = (uint32_t)lane;
    P = pos[nb_ids[o0 + (e < last ? e : last)]];
    const uint32_t e2 = (uint32_t)kTile + e;
    nid = nb_ids[o0 + (e2 < last ? e2 : last)];
  }
  for (uint32_t tb = 0; tb < n; tb += (uint32_t)kTile) {
    __syncthreads();
    tile[lane] = make_float4((float)(P.x - cg.x), (float)(P.y - cg.y),
                             (float)(P.z - cg.z), (float)P.w);
    const uint32_t nb = tb + (uint32_t)kTile;
    if (nb < n) {
      P = pos[nid];
      const uint32_t e = nb + (uint32_t)kTile + (uint32_t)lane;
      nid = nb_ids[o0 + (e < last ? e : last)];
    }
    __syncthreads();
    if (act) {
      const int valid = n - tb < (uint32_t)kTile ? (int)(n - tb) : kTile;
      const int hi = blk1 < valid ? blk1 : valid;
#pragma unroll 8
      for (int k = blk0; k < hi; ++k) {
        const float4 j = tile[k];
        const float dx = j.x - xi, dy = j.y - yi, dz = j.z - zi;
        const float q2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx)) * h2inv;
        if (q2 < 1.f) {
          const float q = __builtin_sqrtf(q2);
          const float u = 1.f - q;
          const float wq =
              q <= 0.5f ? fmaf(6.f * q2, q - 1.f, 1.f) : 2.f * u * u * u;
          sum = fmaf(j.w, wq, sum);
        }
      }
    }
  }
  if (r > 1) {
    __syncthreads();
    red[lane] = sum;
    __syncthreads();
    if (lane < ni) {
      sum = 0.f;
      for (int s2 = 0; s2 < r; ++s2) sum += red[s2 * ni + lane];
    }
  }
  if (lane < ni) rho[it.y + lane] = norm * sum;
}

__global__ void k_zero_queue(unsigned int* q) {
  if (threadIdx.x < 8) q[threadIdx.x] = 0u;
}

// Instance selection: the largest tile (64-entry blocks) and the occupancy
// target the configuration asks for (0 = the defaults above).  The
// persistent launch keeps its own shape.
int force_slices(const nb_ctx* c) {
  const int o = c->cfg.order == 2 ? 2 : 1;
  if ((c->cfg.flags & NB_FLAG_PERSISTENT) || c->cfg.tile_j <= 0)
    return kDefaultSlices[o];
  return c->cfg.tile_j / kTile;
}

int force_waves(const nb_ctx* c) {
  return c->cfg.waves_per_simd > 0 ? c->cfg.waves_per_simd : kDefaultWaves;
}

using ForceFn = void (*)(const uint4*, XcdPlan, ForceArgs);

template <int O, bool C, int K>
ForceFn pick_waves(int waves) {
  switch (waves) {
    case 4: return k_force<O, C, K, 4>;
    case 8: return k_force<O, C, K, 8>;
    default: return k_force<O, C, K, kDefaultWaves>;
  }
}

template <int O, bool C>
ForceFn pick_force(int slices, int waves) {
  switch (slices) {
    case 1: return pick_waves<O, C, 1>(waves);
    case 2: return pick_waves<O, C, 2>(waves);
    case 4: return pick_waves<O, C, 4>(waves);
    default: return pick_waves<O, C, 3>(waves);
  }
}

using CostFn = void (*)(int64_t, const uint32_t*, const uint4*,
                        const uint32_t*, const uint32_t*, uint32_t*);
using TailFn = void (*)(const uint4*, const uint32_t*, const uint32_t*,
                        XcdPlan, uint32_t*);

template <int WS>
CostFn pick_cost(int slices) {
  switch (slices) {
    case 1: return k_group_cost<1, WS>;
    case 2: return k_group_cost<2, WS>;
    case 4: return k_group_cost<4, WS>;
    default: return k_group_cost<3, WS>;
  }
}

template <int WS>
TailFn pick_tail(int slices) {
  switch (slices) {
    case 1: return k_tail_order<1, WS>;
    case 2: return k_tail_order<2, WS>;
    case 4: return k_tail_order<4, WS>;
    default: return k_tail_order<3, WS>;
  }
}

}  // namespace

int launch_force(nb_ctx* c) {
  int rc = reserve(c, c->acc, (size_t)c->n);
  if (rc) return rc;
  if (c->n_wi <= 0) return NB_OK;
  const int64_t per_xcd = (c->n_wi + 7) / 8;
  if (per_xcd * 8 > 0x7FFFFFFFLL)
    return set_err(c, NB_ERR_INPUT, "too many force work items");
  // the plan of the last list construction, with its tail order when that
  // was made for the same plan
  XcdPlan plan;
  const int64_t nblk = checked_plan(c->n_wi, c->xcd_b, plan);
  use_tail(c->tail, plan);
  if (nblk > 0x7FFFFFFFLL)
    return set_err(c, NB_ERR_INPUT, "too many force work items");
  ForceArgs A;
  A.g_cell = c->g_cell.p;
  A.rec = c->c_rec.p;
  A.epj_off = c->epj_off.p;
  A.epj = c->epj.p;
  A.spj_off = c->spj_off.p;
  A.spj = c->spj.p;
  A.cnt_e = c->cnt_e.p;
  A.cnt_s = c->cnt_s.p;
  A.pos = c->pos.p;
  A.pm = c->c_pm.p;
  A.quad = c->c_quad.p;
  A.jcopy = nullptr;
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
                       (const uint4*)c->wi.p, plan, c->queue.p, A);
  } else if (c->cfg.flags & NB_FLAG_COPIED_LISTS) {
    // monopole only (checked with the configuration)
    if ((rc = reserve(c, c->jcopy, (size_t)(c->n_epj + c->n_spj) + 1)))
      return rc;
    const int64_t cblk = grid_for(c->n_groups, 4);
    hipLaunchKernelGGL(k_copy_j, dim3((unsigned)((cblk + 7) / 8 * 8)),
                       dim3(256), 0, c->stream, c->n_groups, cblk,
                       (const uint32_t*)c->g_cell.p,
                       (const CellRec*)c->c_rec.p,
                       (const uint64_t*)c->epj_off.p,
                       (const uint32_t*)c->epj.p,
                       (const uint64_t*)c->spj_off.p,
                       (const uint32_t*)c->spj.p, (const double4*)c->pos.p,
                       (const double4*)c->c_pm.p, c->jcopy.p);
    A.jcopy = c->jcopy.p;
    const ForceFn kc = pick_force<1, true>(force_slices(c), force_waves(c));
    hipLaunchKernelGGL(kc, dim3((unsigned)nblk), dim3(kTile), 0, c->stream,
                       (const uint4*)c->wi.p, plan, A);
  } else {
    const int ks = force_slices(c), kw = force_waves(c);
    ForceFn k = c->cfg.order == 2 ? pick_force<2, false>(ks, kw)
                                  : pick_force<1, false>(ks, kw);
    hipLaunchKernelGGL(k, dim3((unsigned)nblk), dim3(kTile), 0, c->stream,
                       (const uint4*)c->wi.p, plan, A);
  }
  return hip_check(c, hipGetLastError(), "force launch");
}

// Longest-first order of the tail of every XCD's stretch of the force
// launch, from the plan read back with the list totals.
int launch_tail_order(nb_ctx* c) {
  TailOrder& t = c->tail;
  t.valid = false;
  if (c->n_wi <= 0) return NB_OK;
  XcdPlan plan;
  (void)checked_plan(c->n_wi, c->xcd_b, plan);
  for (int x = 0; x < 8; ++x)
    plan.ws[x] = std::max(plan.b[x], plan.b[x + 1] - (int64_t)kTailItems);
  int rc = reserve(c, t.order, 8 * (size_t)kTailItems);
  if (rc) return rc;
  TailFn k = c->cfg.order == 2 ? pick_tail<2>(force_slices(c))
                                : pick_tail<1>(force_slices(c));
  hipLaunchKernelGGL(k, dim3(8), dim3(1024), 0, c->stream,
                     (const uint4*)c->wi.p, (const uint32_t*)c->cnt_e.p,
                     (const uint32_t*)c->cnt_s.p, plan, t.order.p);
  rc = hip_check(c, hipGetLastError(), "tail order launch");
  if (rc) return rc;
  std::copy(plan.b, plan.b + 9, t.b);
  t.valid = true;
  return NB_OK;
}

// Plan of the force launch (or, `neighbours`, of the SPH density launch)
// from the lists just made, before their totals are read back: the nine
// item indices come back with them.
int launch_xcd_plan(nb_ctx* c, bool neighbours) {
  const size_t ng = (size_t)c->n_groups;
  int rc = reserve(c, c->g_cost, ng);
  if (!rc) rc = reserve(c, c->g_cost_off, ng + 1);
  if (!rc) rc = reserve(c, c->xcd_plan, 9);
  if (rc) return rc;
  CostFn k = neighbours ? k_group_cost<1, 1>
                        : (c->cfg.order == 2 ? pick_cost<2>(force_slices(c))
                                             : pick_cost<1>(force_slices(c)));
  hipLaunchKernelGGL(k, dim3(grid_for(c->n_groups, 256)), dim3(256), 0,
                     c->stream, c->n_groups, (const uint32_t*)c->g_chunks.p,
                     (const uint4*)c->wi.p,
                     (const uint32_t*)(neighbours ? c->nb_cnt.p : c->cnt_e.p),
                     (const uint32_t*)(neighbours ? nullptr : c->cnt_s.p),
                     c->g_cost.p);
  rc = hip_check(c, hipGetLastError(), "group cost launch");
  if (!rc) rc = scan_u32_to_u64(c, c->g_cost.p, c->g_cost_off.p, c->n_groups);
  if (rc) return rc;
  hipLaunchKernelGGL(k_xcd_split, dim3(1), dim3(64), 0, c->stream,
                     c->n_groups, (const uint64_t*)c->g_cost_off.p,
                     (const uint32_t*)c->g_chunks.p, c->xcd_plan.p);
  return hip_check(c, hipGetLastError(), "plan launch");
}


// SPH density with smoothing length h on the neighbour lists.
int launch_density(nb_ctx* c, double h) {
  int rc = reserve(c, c->rho, (size_t)c->n);
  if (rc) return rc;
  if (c->n_wi <= 0) return NB_OK;
  XcdPlan plan;
  const int64_t nblk = checked_plan(c->n_wi, c->nbr_b, plan);
  if (nblk > 0x7FFFFFFFLL)
    return set_err(c, NB_ERR_INPUT, "too many work items");
  const double pi = 3.14159265358979323846;
  hipLaunchKernelGGL(k_density, dim3((unsigned)nblk), dim3(kTile), 0,
                     c->stream, (const uint4*)c->wi.p, plan,
                     (const uint32_t*)c->g_cell.p, (const CellRec*)c->c_rec.p,
                     (const uint64_t*)c->nb_off.p,
                     (const uint32_t*)c->nb_ids.p, (const double4*)c->pos.p,
                     (float)(1.0 / (h * h)), (float)(8.0 / (pi * h * h * h)),
                     c->rho.p);
  return hip_check(c, hipGetLastError(), "density launch");
}

}  // namespace nb
