// nb_tree.hip -- construction step of the local tree on the GPU
// (section 4.3): root cell, Morton keys, reorder, link, moments, groups.
//
// Compiled with -ffp-contract=off: the root cube, the keys, the cell centres
// and the group boxes must come out bit-identical to a plain FP64 reference.
//
// Link without a per-level loop.  With keys sorted, the level-l cell holding
// particle i has more than n_leaf particles iff some window of n_leaf + 1
// consecutive keys that covers i shares its first l digits.  So the leaf
// level of i is lam(i) = min(21, 1 + max over windows covering i of the
// digits shared by the window's end keys), and the cells that begin at i are
// the levels lmin(i)..lam(i), where lmin(i) is one more than the digits i
// shares with i-1.  An exclusive scan of lam - lmin + 1 numbers every cell in
// DFS pre-order (sorted by begin, then level); the end of a cell is found by
// a galloping search in the sorted keys (the paper's binary search), and the
// first cell starting at or after that end is the cell after its subtree.
#include <algorithm>

#include "nb_internal.h"

namespace nb {
namespace {

// --- Morton helpers: 21 bits per axis, x most significant in every digit ---
__device__ inline uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

__device__ inline uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
}

// Number of leading 3-bit digits two 63-bit keys share (21 if equal).
__device__ inline int shared_levels(uint64_t a, uint64_t b) {
  const uint64_t d = a ^ b;
  if (d == 0) return kMaxLevel;
  return (__clzll((long long)d) - 1) / 3;
}

// ---------------------------------------------------------------------------
// Root cell: per-axis min / max of the positions (exact), then the cube.
constexpr int kBboxThreads = 256;

__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Per-chunk partials; a chunk lies inside one system.
__global__ void __launch_bounds__(kBboxThreads)
k_bbox_partial(const double4* __restrict__ pos,
               const int4* __restrict__ chunks, double* __restrict__ part) {
  __shared__ double s[kBboxThreads / 64][7];
  const int4 ch = chunks[blockIdx.x];
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  double bad = 0.0;
  for (int64_t i = (int64_t)ch.y + threadIdx.x; i < (int64_t)ch.z;
       i += blockDim.x) {
    const double4 p = pos[i];
    const double v[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (!isfinite(v[a])) bad = 1.0;
      mn[a] = fmin(mn[a], v[a]);
      mx[a] = fmax(mx[a], v[a]);
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double r[7];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = wave_min(mn[a]);
    r[3 + a] = wave_max(mx[a]);
  }
  r[6] = wave_max(bad);
  if (lane == 0)
    for (int a = 0; a < 7; ++a) s[w][a] = r[a];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kBboxThreads / 64; ++q) {
      for (int a = 0; a < 3; ++a) {
        s[0][a] = fmin(s[0][a], s[q][a]);
        s[0][3 + a] = fmax(s[0][3 + a], s[q][3 + a]);
      }
      s[0][6] = fmax(s[0][6], s[q][6]);
    }
    for (int a = 0; a < 7; ++a) part[(int64_t)blockIdx.x * 8 + a] = s[0][a];
  }
}

// rr = (1/theta)*(1/theta) from the host: (2^e/theta)^2 rounds to
// 2^(2e) * rr exactly, so rcrit2[l] = ldexp(rr, 2(k - l)).
// One block of 256 threads per system reduces that system's chunk partials
// (min / max are exact, so the reduction order does not matter).
__global__ void __launch_bounds__(kBboxThreads)
k_bbox_final(const double* __restrict__ part,
             const uint32_t* __restrict__ first, double rr,
             Root* __restrict__ roots) {
  __shared__ double s[kBboxThreads / 64][7];
  const uint32_t b0 = first[blockIdx.x], b1 = first[blockIdx.x + 1];
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  double bad = 0.0;
  for (uint32_t b = b0 + threadIdx.x; b < b1; b += kBboxThreads) {
    for (int a = 0; a < 3; ++a) {
      mn[a] = fmin(mn[a], part[(int64_t)b * 8 + a]);
      mx[a] = fmax(mx[a], part[(int64_t)b * 8 + 3 + a]);
    }
    bad = fmax(bad, part[(int64_t)b * 8 + 6]);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int a = 0; a < 3; ++a) {
    mn[a] = wave_min(mn[a]);
    mx[a] = wave_max(mx[a]);
  }
  bad = wave_max(bad);
  if (lane == 0) {
    for (int a = 0; a < 3; ++a) {
      s[w][a] = mn[a];
      s[w][3 + a] = mx[a];
    }
    s[w][6] = bad;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int q = 1; q < kBboxThreads / 64; ++q) {
    for (int a = 0; a < 3; ++a) {
      s[0][a] = fmin(s[0][a], s[q][a]);
      s[0][3 + a] = fmax(s[0][3 + a], s[q][3 + a]);
    }
    s[0][6] = fmax(s[0][6], s[q][6]);
  }
  Root* root = roots + blockIdx.x;
  double ext = 0.0;
  for (int a = 0; a < 3; ++a) {
    root->lo[a] = s[0][a];
    const double e = s[0][3 + a] - s[0][a];
    if (e > ext) ext = e;
  }
  int k = 0;
  if (ext > 0.0 && isfinite(ext)) {
    frexp(ext, &k);
    while (ldexp(1.0, k) <= ext) k++;
    while (ldexp(1.0, k - 1) > ext) k--;
  }
  root->k = k;
  root->rr = rr;
  root->bad = (s[0][6] != 0.0 || !isfinite(ext)) ? 1 : 0;
  for (int l = 0; l < kLevels; ++l) root->rcrit2[l] = ldexp(rr, 2 * (k - l));
}

// Any system with a non-finite coordinate -> roots[0].bad (read by the host).
__global__ void k_bbox_bad(Root* __restrict__ roots, int64_t n_sys) {
  if (threadIdx.x != 0) return;
  int bad = 0;
  for (int64_t s = 0; s < n_sys; ++s) bad |= roots[s].bad;
  roots[0].bad = bad;
}

// ---------------------------------------------------------------------------
// Morton keys: q = floor((x - lo) * 2^(21 - k)), clamped to 21 bits.
__global__ void __launch_bounds__(256)
k_keys(const double4* __restrict__ pos, int64_t n,
       const Root* __restrict__ roots, const uint32_t* __restrict__ seg,
       uint64_t* __restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Root* root = roots + seg[i];
  const double scale = ldexp(1.0, kKeyBits - root->k);
  const double qmax = (double)((1u << kKeyBits) - 1u);
  const double4 p = pos[i];
  const double v[3] = {p.x, p.y, p.z};
  uint32_t q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double d = __dsub_rn(v[a], root->lo[a]);
    double f = floor(__dmul_rn(d, scale));
    f = f < 0.0 ? 0.0 : (f > qmax ? qmax : f);
    q[a] = (uint32_t)f;
  }
  key[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
}

// Reorder: gather the particle state into Morton order (section 4.3, local
// tree step 3).  val holds, per sorted slot, the slot it came from.
__global__ void __launch_bounds__(256)
k_gather(int64_t n, const uint32_t* __restrict__ val,
         const double4* __restrict__ pos, const double* __restrict__ vx,
         const double* __restrict__ vy, const double* __restrict__ vz,
         const uint32_t* __restrict__ orig, double4* __restrict__ pos2,
         double* __restrict__ vx2, double* __restrict__ vy2,
         double* __restrict__ vz2, uint32_t* __restrict__ orig2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = val[i];
  pos2[i] = pos[s];
  vx2[i] = vx[s];
  vy2[i] = vy[s];
  vz2[i] = vz[s];
  orig2[i] = orig[s];
}

// ---------------------------------------------------------------------------
// Link, pass 1: leaf level lam(i), first level lmin(i) of a cell beginning
// at i, and the number of cells beginning at i.
// Link, pass 1: leaf level lam(i), first level lmin(i) of a cell beginning
// at i, and the number of cells beginning at i.  Windows and neighbours
// never reach across the particle's system: each system has its own root.
__global__ void __launch_bounds__(256)
k_link_count(const uint64_t* __restrict__ key, int64_t n, int n_leaf,
             const uint32_t* __restrict__ seg,
             const uint32_t* __restrict__ sys_off,
             uint8_t* __restrict__ lam, uint8_t* __restrict__ lmin,
             uint32_t* __restrict__ cstart) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t si = seg[i];
  const int64_t sb = sys_off[si], se = sys_off[si + 1];
  int M = -1;
  const int64_t s0 = i - n_leaf > sb ? i - n_leaf : sb;
  for (int64_t s = s0; s <= i; ++s) {
    if (s + n_leaf < se) {
      const int v = shared_levels(key[s], key[s + n_leaf]);
      M = v > M ? v : M;
    }
  }
  const int la = M < 0 ? 0 : (M + 1 < kMaxLevel ? M + 1 : kMaxLevel);
  const int lm = i == sb ? 0 : shared_levels(key[i - 1], key[i]) + 1;
  lam[i] = (uint8_t)la;
  lmin[i] = (uint8_t)lm;
  cstart[i] = la >= lm ? (uint32_t)(la - lm + 1) : 0u;
}

// First index >= lo whose key differs from `pre` in its top digits
// (keys[lo-1] shares them).
__device__ inline int64_t gallop_end(const uint64_t* __restrict__ key,
                                     int64_t n, int64_t lo, uint64_t pre,
                                     int sh) {
  int64_t a = lo, b = n, step = 1;
  for (;;) {
    const int64_t probe = a + step - 1;
    if (probe >= n) {
      b = n;
      break;
    }
    if ((key[probe] >> sh) != pre) {
      b = probe;
      break;
    }
    a = probe + 1;
    step <<= 1;
  }
  while (a < b) {
    const int64_t mid = a + ((b - a) >> 1);
    if ((key[mid] >> sh) == pre)
      a = mid + 1;
    else
      b = mid;
  }
  return a;
}

// First index in [lo_bound, hi] whose key shares `pre` (keys[hi] does).
__device__ inline int64_t gallop_begin(const uint64_t* __restrict__ key,
                                       int64_t lo_bound, int64_t hi,
                                       uint64_t pre, int sh) {
  int64_t in = hi, out = lo_bound - 1, step = 1;
  for (;;) {
    const int64_t probe = in - step;
    if (probe < lo_bound) {
      out = lo_bound - 1;
      break;
    }
    if ((key[probe] >> sh) != pre) {
      out = probe;
      break;
    }
    in = probe;
    step <<= 1;
  }
  while (in - out > 1) {
    const int64_t mid = out + ((in - out) >> 1);
    if ((key[mid] >> sh) == pre)
      in = mid;
    else
      out = mid;
  }
  return in;
}

// Link, pass 2: write every cell (DFS pre-order id = S[i] + l - lmin(i)).
__global__ void __launch_bounds__(256)
k_link_fill(const uint64_t* __restrict__ key, int64_t n,
            const uint32_t* __restrict__ seg,
            const uint32_t* __restrict__ sys_off,
            const uint8_t* __restrict__ lam, const uint8_t* __restrict__ lmin,
            const uint32_t* __restrict__ S, const Root* __restrict__ roots,
            CellRec* __restrict__ rec, uint4* __restrict__ wrec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int la = lam[i], lm = lmin[i];
  if (la < lm) return;
  const uint32_t si = seg[i];
  const int64_t sb = sys_off[si], se = sys_off[si + 1];
  const Root* root = roots + si;
  const uint32_t base = S[i];
  const uint64_t ki = key[i];
  const int k = root->k;
  int64_t end = i + 1;
  for (int l = la; l >= lm; --l) {
    const uint32_t id = base + (uint32_t)(l - lm);
    const int sh = 3 * (kMaxLevel - l);
    const uint64_t pre = ki >> sh;
    end = gallop_end(key, se, end, pre, sh);
    uint32_t par;
    if (l > lm) {
      par = id - 1;
    } else if (l == 0) {
      par = kNone;
    } else {
      const int psh = 3 * (kMaxLevel - (l - 1));
      const int64_t b = gallop_begin(key, sb, i, ki >> psh, psh);
      par = S[b] + (uint32_t)((l - 1) - (int)lmin[b]);
    }
    const uint32_t skip = S[end];
    // geometric centre: lo + (2q + 1) * 2^(k - l - 1)
    const double half = ldexp(1.0, k - l - 1);
    const uint32_t qx = compact3(pre >> 2), qy = compact3(pre >> 1),
                   qz = compact3(pre);
    CellRec r;
    r.geo.x = __dadd_rn(root->lo[0], __dmul_rn(2.0 * (double)qx + 1.0, half));
    r.geo.y = __dadd_rn(root->lo[1], __dmul_rn(2.0 * (double)qy + 1.0, half));
    r.geo.z = __dadd_rn(root->lo[2], __dmul_rn(2.0 * (double)qz + 1.0, half));
    r.geo.w = root->rcrit2[l];
    r.meta = make_uint4((uint32_t)i, (uint32_t)end, skip,
                        (uint32_t)l | (l == la ? 256u : 0u));
    r.aux = make_uint4(par, 0u, 0u, 0u);
    rec[id] = r;
    const uint64_t q = (uint64_t)qx | ((uint64_t)qy << 21) |
                       ((uint64_t)qz << 42);
    const bool leaf = l == la;
    uint64_t cnt = leaf ? (uint64_t)(end - i) : 0;
    if (cnt > kWalkCountSat) cnt = kWalkCountSat;
    wrec[id] = make_uint4((uint32_t)q,
                          (uint32_t)(q >> 32) | (leaf ? 0x80000000u : 0u),
                          skip, (uint32_t)l | ((uint32_t)cnt << 5));
  }
}

// First cell of every system (its root) and the total: croot[s] = S[off_s].
__global__ void k_sys_roots(const uint32_t* __restrict__ S,
                            const uint32_t* __restrict__ sys_off,
                            int64_t n_sys, uint32_t* __restrict__ croot) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s <= n_sys) croot[s] = S[sys_off[s]];
}

// System of every slot from the system offsets.
__global__ void __launch_bounds__(256)
k_seg_fill(const uint32_t* __restrict__ sys_off, int64_t n_sys, int64_t n,
           uint32_t* __restrict__ seg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t lo = 0, hi = n_sys;  // last s with sys_off[s] <= i
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)sys_off[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  seg[i] = (uint32_t)lo;
}

// ---------------------------------------------------------------------------
// Groups (Barnes' vectorisation): a cell holding at most n_grp particles (or
// a leaf) whose parent holds more than n_grp.
__global__ void __launch_bounds__(256)
k_group_flags(int64_t n_cell, const CellRec* __restrict__ rec, int n_grp,
              uint32_t* __restrict__ gflag) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cell) return;
  const uint4 m = rec[c].meta;
  const uint32_t cnt = m.y - m.x;
  const bool leaf = (m.w >> 8) & 1u;
  bool top = true;  // a system's root has no parent
  if ((m.w & 255u) != 0) {
    const uint4 pm = rec[rec[c].aux.x].meta;
    top = (pm.y - pm.x) > (uint32_t)n_grp;
  }
  gflag[c] = ((cnt <= (uint32_t)n_grp || leaf) && top) ? 1u : 0u;
}

// Cells grouped by level (bucket kLevels = leaves) with a counting sort:
// per-block histograms in LDS, a scan over (bucket, block), then a scatter.
// The order inside a bucket is irrelevant: each cell's moments only need
// its children, which sit one level deeper.
constexpr int kBuckets = kLevels + 1;
constexpr int kBkThreads = 256;
constexpr int kBkItems = 4;
constexpr int kBkTile = kBkThreads * kBkItems;

__device__ inline uint32_t bucket_of(uint32_t w) {
  return ((w >> 8) & 1u) ? (uint32_t)kLevels : (w & 255u);
}

__global__ void __launch_bounds__(kBkThreads)
k_bucket_hist(int64_t n_cell, const CellRec* __restrict__ rec,
              uint32_t* __restrict__ hist, int nblk) {
  __shared__ uint32_t h[kBuckets];
  if (threadIdx.x < kBuckets) h[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kBkItems; ++j) {
    const int64_t c = (int64_t)blockIdx.x * kBkTile + j * kBkThreads + threadIdx.x;
    if (c < n_cell) atomicAdd(&h[bucket_of(rec[c].meta.w)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kBuckets)
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kBkThreads)
k_bucket_scatter(int64_t n_cell, const CellRec* __restrict__ rec,
                 const uint32_t* __restrict__ hist, int nblk,
                 uint32_t* __restrict__ out) {
  __shared__ uint32_t base[kBuckets];
  __shared__ uint32_t cnt[kBuckets];
  if (threadIdx.x < kBuckets) {
    base[threadIdx.x] = hist[(int64_t)threadIdx.x * nblk + blockIdx.x];
    cnt[threadIdx.x] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kBkItems; ++j) {
    const int64_t c = (int64_t)blockIdx.x * kBkTile + j * kBkThreads + threadIdx.x;
    if (c < n_cell) {
      const uint32_t b = bucket_of(rec[c].meta.w);
      out[base[b] + atomicAdd(&cnt[b], 1u)] = (uint32_t)c;
    }
  }
}

// Bucket starts and the group count, gathered for one host read.
__global__ void k_bucket_starts(const uint32_t* __restrict__ hist, int nblk,
                                const uint32_t* __restrict__ gflag,
                                int64_t n_cell, uint32_t* __restrict__ out) {
  const int t = threadIdx.x;
  if (t < kBuckets) out[t] = hist[(int64_t)t * nblk];
  if (t == kBuckets) out[t] = gflag[n_cell];
}

// Chunks of a group for the force kernel: whole 64-particle chunks, then the
// remainder split as the table says (see chunk_table()).
struct ChunkTable {
  uint32_t e[64];  // remainder n: count << 24 | size0 | size1 << 8 | size2 << 16
};

__global__ void __launch_bounds__(256)
k_group_fill(int64_t n_cell, const uint32_t* __restrict__ gscan,
             const CellRec* __restrict__ rec, ChunkTable tab,
             uint32_t* __restrict__ g_cell, uint32_t* __restrict__ g_begin,
             uint32_t* __restrict__ g_count, uint32_t* __restrict__ chunks) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cell) return;
  const uint32_t g = gscan[c];
  if (gscan[c + 1] == g) return;
  const uint4 m = rec[c].meta;
  const uint32_t n = m.y - m.x;
  g_cell[g] = (uint32_t)c;
  g_begin[g] = m.x;
  g_count[g] = n;
  chunks[g] = n / 64u + (tab.e[n % 64u] >> 24);
}

// One wave per group: exact FP64 min / max of the member positions.
__global__ void __launch_bounds__(256)
k_group_box(int64_t n_groups, const uint32_t* __restrict__ g_begin,
            const uint32_t* __restrict__ g_count,
            const double4* __restrict__ pos, double4* __restrict__ g_lo,
            double4* __restrict__ g_hi) {
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= n_groups) return;
  const uint32_t b = g_begin[g], cnt = g_count[g];
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (uint32_t j = lane; j < cnt; j += 64) {
    const double4 p = pos[b + j];
    mn[0] = fmin(mn[0], p.x);
    mn[1] = fmin(mn[1], p.y);
    mn[2] = fmin(mn[2], p.z);
    mx[0] = fmax(mx[0], p.x);
    mx[1] = fmax(mx[1], p.y);
    mx[2] = fmax(mx[2], p.z);
  }
  for (int a = 0; a < 3; ++a) {
    mn[a] = wave_min(mn[a]);
    mx[a] = wave_max(mx[a]);
  }
  if (lane == 0) {
    g_lo[g] = make_double4(mn[0], mn[1], mn[2], 0.0);
    g_hi[g] = make_double4(mx[0], mx[1], mx[2], 0.0);
  }
}

__global__ void __launch_bounds__(256)
k_make_wi(int64_t n_groups, const uint32_t* __restrict__ g_begin,
          const uint32_t* __restrict__ g_count, ChunkTable tab,
          const uint32_t* __restrict__ choff, uint4* __restrict__ wi) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  uint32_t b = g_begin[g];
  const uint32_t cnt = g_count[g];
  uint32_t o = choff[g];
  for (uint32_t s = 0; s + 64u <= cnt; s += 64u, ++o, b += 64u)
    wi[o] = make_uint4((uint32_t)g, b, 64u, 0u);
  const uint32_t t = tab.e[cnt % 64u];
  for (uint32_t k = 0; k < (t >> 24); ++k, ++o) {
    const uint32_t len = (t >> (8 * k)) & 255u;
    wi[o] = make_uint4((uint32_t)g, b, len, 0u);
    b += len;
  }
}

// ---------------------------------------------------------------------------
// Moments (section 4.3: recomputed at every step, reuse steps included).
// Offsets from the cell's geometric centre are formed in FP64 and kept in
// FP32; parents combine their children with the parallel-axis rule in FP32
// (the child-to-parent centre shift is an exact power of two).
// Leaves: four lanes per leaf, lane s taking particles s, s + 4, ... of it,
// so that the lanes of a wave read consecutive particles; the four partial
// sums are combined pairwise across the lanes.
constexpr int kLeafLanes = 4;

__device__ inline float sum_leaf_lanes(float v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  return v;
}

template <bool QUAD>
__global__ void __launch_bounds__(256)
k_mom_leaf(int64_t cnt, const uint32_t* __restrict__ list,
           const CellRec* __restrict__ rec, const double4* __restrict__ pos,
           float4* __restrict__ mom, float4* __restrict__ quad,
           double4* __restrict__ pm) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t = gt / kLeafLanes;
  const uint32_t s = (uint32_t)(gt % kLeafLanes);
  // the lanes of one leaf leave together, so the exchanges below only
  // involve lanes that are still running
  if (t >= cnt) return;
  const uint32_t c = list[t];
  const uint4 m = rec[c].meta;
  const double4 g = rec[c].geo;
  float M = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
  for (uint32_t p = m.x + s; p < m.y; p += kLeafLanes) {
    const double4 P = pos[p];
    const float w = (float)P.w;
    const float dx = (float)(P.x - g.x), dy = (float)(P.y - g.y),
                dz = (float)(P.z - g.z);
    M += w;
    sx = fmaf(w, dx, sx);
    sy = fmaf(w, dy, sy);
    sz = fmaf(w, dz, sz);
  }
  M = sum_leaf_lanes(M);
  sx = sum_leaf_lanes(sx);
  sy = sum_leaf_lanes(sy);
  sz = sum_leaf_lanes(sz);
  const float inv = M > 0.f ? 1.0f / M : 0.f;
  const float ox = sx * inv, oy = sy * inv, oz = sz * inv;
  if (s == 0) {
    mom[c] = make_float4(ox, oy, oz, M);
    pm[c] = make_double4(g.x + (double)ox, g.y + (double)oy,
                         g.z + (double)oz, (double)M);
  }
  if (QUAD) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f;
    for (uint32_t p = m.x + s; p < m.y; p += kLeafLanes) {
      const double4 P = pos[p];
      const float w = (float)P.w;
      const float dx = (float)(P.x - g.x) - ox, dy = (float)(P.y - g.y) - oy,
                  dz = (float)(P.z - g.z) - oz;
      s0 = fmaf(w * dx, dx, s0);
      s1 = fmaf(w * dy, dy, s1);
      s2 = fmaf(w * dz, dz, s2);
      s3 = fmaf(w * dx, dy, s3);
      s4 = fmaf(w * dx, dz, s4);
      s5 = fmaf(w * dy, dz, s5);
    }
    s0 = sum_leaf_lanes(s0);
    s1 = sum_leaf_lanes(s1);
    s2 = sum_leaf_lanes(s2);
    s3 = sum_leaf_lanes(s3);
    s4 = sum_leaf_lanes(s4);
    s5 = sum_leaf_lanes(s5);
    if (s == 0) {
      quad[2 * (int64_t)c] = make_float4(s0, s1, s2, s3);
      quad[2 * (int64_t)c + 1] = make_float4(s4, s5, 0.f, 0.f);
    }
  }
}

// Next sibling; a skip id that does not advance ends the loop.
__device__ inline uint32_t next_child(const CellRec* __restrict__ rec,
                                      uint32_t k, uint32_t stop) {
  const uint32_t s = rec[k].meta.z;
  return s > k ? s : stop;
}

template <bool QUAD>
__global__ void __launch_bounds__(256)
k_mom_internal(int64_t cnt, const uint32_t* __restrict__ list,
               const CellRec* __restrict__ rec, float4* __restrict__ mom,
               float4* __restrict__ quad, double4* __restrict__ pm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const uint32_t c = list[t];
  const uint32_t stop = rec[c].meta.z;
  const double4 g = rec[c].geo;
  float M = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
  for (uint32_t k = c + 1; k < stop; k = next_child(rec, k, stop)) {
    const float4 mk = mom[k];
    const double4 gk = rec[k].geo;
    const float dx = (float)(gk.x - g.x) + mk.x;
    const float dy = (float)(gk.y - g.y) + mk.y;
    const float dz = (float)(gk.z - g.z) + mk.z;
    M += mk.w;
    sx = fmaf(mk.w, dx, sx);
    sy = fmaf(mk.w, dy, sy);
    sz = fmaf(mk.w, dz, sz);
  }
  const float inv = M > 0.f ? 1.0f / M : 0.f;
  const float ox = sx * inv, oy = sy * inv, oz = sz * inv;
  mom[c] = make_float4(ox, oy, oz, M);
  pm[c] = make_double4(g.x + (double)ox, g.y + (double)oy, g.z + (double)oz,
                       (double)M);
  if (QUAD) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f;
    for (uint32_t k = c + 1; k < stop; k = next_child(rec, k, stop)) {
      const float4 mk = mom[k];
      const double4 gk = rec[k].geo;
      const float4 qa = quad[2 * (int64_t)k];
      const float4 qb = quad[2 * (int64_t)k + 1];
      const float dx = (float)(gk.x - g.x) + mk.x - ox;
      const float dy = (float)(gk.y - g.y) + mk.y - oy;
      const float dz = (float)(gk.z - g.z) + mk.z - oz;
      const float w = mk.w;
      s0 += qa.x + w * dx * dx;
      s1 += qa.y + w * dy * dy;
      s2 += qa.z + w * dz * dz;
      s3 += qa.w + w * dx * dy;
      s4 += qb.x + w * dx * dz;
      s5 += qb.y + w * dy * dz;
    }
    quad[2 * (int64_t)c] = make_float4(s0, s1, s2, s3);
    quad[2 * (int64_t)c + 1] = make_float4(s4, s5, 0.f, 0.f);
  }
}

// ---------------------------------------------------------------------------
// Moments in two launches instead of one per level.  A block is a maximal
// subtree of at most kMomBlock cells (its cells are a contiguous stretch of
// the pre-order array); one workgroup computes a block bottom-up in LDS,
// leaves from their particles, then one level per barrier, and writes the
// block's moments out at the end.  The cells above the blocks (subtrees of
// more than kMomBlock cells, the "top" cells) are then summed by a single
// workgroup, level by level, through a table of eight children by octant
// per top cell: a block's root leaves the terms it adds to its parent's sums
// in its slot of that table, and top children are exchanged through LDS.
// Every cell's sums are formed
// in the same order and precision as the per-level kernels above (leaves:
// four interleaved partial sums added pairwise; internal cells: children in
// pre-order), so the moments are the same bit for bit.
constexpr int kMomBlock = 1024;
constexpr int kMomThreads = 256;
constexpr int kMomPer = kMomBlock / kMomThreads;
constexpr int kMomTopThreads = 1024;
// top cells kept in LDS by the top launch, monopole (half with quadrupoles;
// more: it works from global memory); the child table marks a child that is
// a top cell with kTopTag and its position in the top list
constexpr int kMomTopLds = 2048;
constexpr uint32_t kTopTag = 0x80000000u;
// particles of a leaf loaded together
constexpr int kLeafChunk = 4;

__device__ inline uint32_t subtree_cells(const uint4 m, uint32_t c) {
  return m.z - c;  // the skip id is always past the cell
}

// Octant of a cell inside its parent, from its integer coordinates in the
// walk record (x the high bit, as in the keys): children in octant order
// are children in pre-order.
__device__ inline uint32_t cell_octant(const uint4 w) {
  const uint64_t q = (uint64_t)w.x | ((uint64_t)(w.y & 0x7FFFFFFFu) << 32);
  return (uint32_t)(((q & 1u) << 2) | (((q >> 21) & 1u) << 1) |
                    ((q >> 42) & 1u));
}

// Block roots: at most kMomBlock cells in the subtree, and a system root or
// a parent with more.
__global__ void __launch_bounds__(256)
k_mp_flags(int64_t n_cell, const CellRec* __restrict__ rec,
           uint32_t* __restrict__ bflag) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cell) return;
  const uint4 m = rec[c].meta;
  bool root = subtree_cells(m, (uint32_t)c) <= (uint32_t)kMomBlock;
  if (root && (m.w & 255u) != 0) {
    const uint32_t p = rec[c].aux.x;
    root = subtree_cells(rec[p].meta, p) > (uint32_t)kMomBlock;
  }
  bflag[c] = root ? 1u : 0u;
}

__global__ void __launch_bounds__(256)
k_mp_blocks(int64_t n_cell, const uint32_t* __restrict__ bscan,
            uint32_t* __restrict__ blocks) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cell) return;
  const uint32_t b = bscan[c];
  if (bscan[c + 1] != b) blocks[b] = (uint32_t)c;
}

// Top cells over the level-sorted cell list (leaves, never top, come last).
__global__ void __launch_bounds__(256)
k_mp_tflags(int64_t n_cell, const uint32_t* __restrict__ lvl,
            const CellRec* __restrict__ rec, uint32_t* __restrict__ tflag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cell) return;
  const uint32_t c = lvl[i];
  tflag[i] = subtree_cells(rec[c].meta, c) > (uint32_t)kMomBlock ? 1u : 0u;
}

// Top list by level (ascending), and each top cell's position in it
// (rec.aux.y), by which the child table is indexed.
__global__ void __launch_bounds__(256)
k_mp_top(int64_t n_cell, const uint32_t* __restrict__ lvl,
         const uint32_t* __restrict__ tscan, uint32_t* __restrict__ top,
         int64_t top_cap, CellRec* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cell) return;
  const uint32_t j = tscan[i];
  if (tscan[i + 1] == j || (int64_t)j >= top_cap) return;
  const uint32_t c = lvl[i];
  top[j] = c;
  rec[c].aux.y = j;
}

// Where each level starts in the top list (tlo[0 .. kLevels]; the level
// buckets start at bstart[0 .. kLevels], leaves last), and the block and top
// counts for the host (stage[0], stage[1]); clears the child table.
__global__ void __launch_bounds__(256)
k_mp_tlo(int64_t n_cell, const uint32_t* __restrict__ bstart,
         const uint32_t* __restrict__ tscan,
         const uint32_t* __restrict__ bscan, uint32_t* __restrict__ tlo,
         uint32_t* __restrict__ stage, uint32_t* __restrict__ ctab,
         int64_t top_cap) {
  // (top_cap bounds the top cells; a count past it would be a broken tree:
  // the list is cut there, so that no launch reads past the buffers)
  const uint32_t n_top = (int64_t)tscan[n_cell] < top_cap
                             ? tscan[n_cell] : (uint32_t)top_cap;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= kLevels) {
    const uint32_t v = tscan[bstart[t] < n_cell ? bstart[t] : n_cell];
    tlo[t] = v < n_top ? v : n_top;
  }
  if (t == 0) {
    stage[0] = bscan[n_cell];
    stage[1] = n_top;
  }
  for (int64_t k = t; k < 8 * (int64_t)n_top;
       k += (int64_t)gridDim.x * blockDim.x)
    ctab[k] = kNone;
}

// Child table of the top cells: slot 8 j + octant of the top cell at
// position j holds that child: its id, or kTopTag | its position when it is
// a top cell itself (kNone: no child there).  The octant comes from the
// child's integer coordinates (x the high bit), so slot order is pre-order.
__global__ void __launch_bounds__(256)
k_mp_ctab(int64_t n_cell, const CellRec* __restrict__ rec,
          const uint4* __restrict__ wrec, uint32_t* __restrict__ ctab,
          int64_t ctab_cap) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cell) return;
  const uint4 m = rec[c].meta;
  if ((m.w & 255u) == 0) return;
  const uint32_t p = rec[c].aux.x;
  if (subtree_cells(rec[p].meta, p) <= (uint32_t)kMomBlock) return;
  const int64_t slot = 8 * (int64_t)rec[p].aux.y + cell_octant(wrec[c]);
  const bool is_top = subtree_cells(m, (uint32_t)c) > (uint32_t)kMomBlock;
  if (slot < ctab_cap)
    ctab[slot] = is_top ? (kTopTag | rec[c].aux.y) : (uint32_t)c;
}

// A leaf's sums from its particles: the four interleaved partial sums of
// k_mom_leaf's lanes (particle i of the leaf goes to sum i % 4), added
// pairwise as its exchanges add them.  The particles are loaded four at a
// time (a leaf of the disk holds 2.8 on average), so that a leaf waits for
// one load latency per four.
template <bool QUAD>
__device__ __forceinline__ void leaf_sums(const uint4 m, const double4 g,
                                          const double4* __restrict__ pos,
                                          float4& mo, float4& qa,
                                          float4& qb) {
  float pM[4] = {0.f, 0.f, 0.f, 0.f}, px[4] = {0.f, 0.f, 0.f, 0.f},
        py[4] = {0.f, 0.f, 0.f, 0.f}, pz[4] = {0.f, 0.f, 0.f, 0.f};
  for (uint32_t b = m.x; b < m.y; b += kLeafChunk) {
    double4 P[kLeafChunk];
#pragma unroll
    for (int i = 0; i < kLeafChunk; ++i)
      P[i] = pos[b + i < m.y ? b + i : m.y - 1];
#pragma unroll
    for (int i = 0; i < kLeafChunk; ++i) {
      if (b + i >= m.y) break;
      const int s = i & (kLeafLanes - 1);
      const float w = (float)P[i].w;
      const float dx = (float)(P[i].x - g.x), dy = (float)(P[i].y - g.y),
                  dz = (float)(P[i].z - g.z);
      pM[s] += w;
      px[s] = fmaf(w, dx, px[s]);
      py[s] = fmaf(w, dy, py[s]);
      pz[s] = fmaf(w, dz, pz[s]);
    }
  }
  const float M = (pM[0] + pM[1]) + (pM[2] + pM[3]);
  const float sx = (px[0] + px[1]) + (px[2] + px[3]);
  const float sy = (py[0] + py[1]) + (py[2] + py[3]);
  const float sz = (pz[0] + pz[1]) + (pz[2] + pz[3]);
  const float inv = M > 0.f ? 1.0f / M : 0.f;
  const float ox = sx * inv, oy = sy * inv, oz = sz * inv;
  mo = make_float4(ox, oy, oz, M);
  if (!QUAD) return;
  float q[6][4];
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int s = 0; s < 4; ++s) q[k][s] = 0.f;
  for (uint32_t b = m.x; b < m.y; b += kLeafChunk) {
    double4 P[kLeafChunk];
#pragma unroll
    for (int i = 0; i < kLeafChunk; ++i)
      P[i] = pos[b + i < m.y ? b + i : m.y - 1];
#pragma unroll
    for (int i = 0; i < kLeafChunk; ++i) {
      if (b + i >= m.y) break;
      const int s = i & (kLeafLanes - 1);
      const float w = (float)P[i].w;
      const float dx = (float)(P[i].x - g.x) - ox,
                  dy = (float)(P[i].y - g.y) - oy,
                  dz = (float)(P[i].z - g.z) - oz;
      q[0][s] = fmaf(w * dx, dx, q[0][s]);
      q[1][s] = fmaf(w * dy, dy, q[1][s]);
      q[2][s] = fmaf(w * dz, dz, q[2][s]);
      q[3][s] = fmaf(w * dx, dy, q[3][s]);
      q[4][s] = fmaf(w * dx, dz, q[4][s]);
      q[5][s] = fmaf(w * dy, dz, q[5][s]);
    }
  }
  float r[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) r[k] = (q[k][0] + q[k][1]) + (q[k][2] + q[k][3]);
  qa = make_float4(r[0], r[1], r[2], r[3]);
  qb = make_float4(r[4], r[5], 0.f, 0.f);
}

// One block per workgroup.  Cell p of the block (id c0 + p) is taken by
// thread p % kMomThreads.  LDS holds per cell its skip id (relative to c0)
// with its level and leaf flag, the FP32 offset of its centre from its
// parent's (the term (float)(child centre - parent centre) of the parent's
// sums, formed in FP64 and rounded once, as k_mom_internal forms it) and its
// moments.  Nothing is written to global memory before the last barrier, so
// the barriers wait for LDS only.
template <bool QUAD>
__global__ void __launch_bounds__(kMomThreads)
k_mom_block(const uint32_t* __restrict__ blocks,
            const CellRec* __restrict__ rec, const uint4* __restrict__ wrec,
            const double4* __restrict__ pos, float4* __restrict__ mom,
            float4* __restrict__ quad, double4* __restrict__ pm,
            float4* __restrict__ slot, int64_t slot_cap) {
  __shared__ uint32_t s_word[kMomBlock];  // skip | level << 16 | leaf << 24
  __shared__ float s_ox[kMomBlock], s_oy[kMomBlock], s_oz[kMomBlock];
  __shared__ float4 s_mom[kMomBlock];
  __shared__ float4 s_q[QUAD ? 2 * kMomBlock : 1];
  __shared__ int s_lmax;
  const uint32_t c0 = blocks[blockIdx.x];
  const int tid = threadIdx.x;
  const uint4 m0 = rec[c0].meta;
  const uint32_t size = subtree_cells(m0, c0);
  if (size > (uint32_t)kMomBlock) return;  // not a block (uniform)
  if (tid == 0) s_lmax = -1;
  __syncthreads();
  int lmax = -1;
  double gx[kMomPer], gy[kMomPer], gz[kMomPer];
#pragma unroll
  for (int u = 0; u < kMomPer; ++u) {
    const uint32_t p = (uint32_t)(u * kMomThreads + tid);
    if (p >= size) continue;
    const uint32_t c = c0 + p;
    const uint4 m = rec[c].meta;
    const double4 g = rec[c].geo;
    gx[u] = g.x;
    gy[u] = g.y;
    gz[u] = g.z;
    const uint32_t lev = m.w & 255u;
    const bool leaf = (m.w >> 8) & 1u;
    s_word[p] = (m.z - c0) | (lev << 16) | (leaf ? (1u << 24) : 0u);
    if (p > 0) {
      const double4 gp = rec[rec[c].aux.x].geo;
      s_ox[p] = (float)(g.x - gp.x);
      s_oy[p] = (float)(g.y - gp.y);
      s_oz[p] = (float)(g.z - gp.z);
    }
    if (!leaf) {
      lmax = (int)lev > lmax ? (int)lev : lmax;
      continue;
    }
    float4 mo, qa, qb;
    leaf_sums<QUAD>(m, g, pos, mo, qa, qb);
    s_mom[p] = mo;
    if (QUAD) {
      s_q[2 * p] = qa;
      s_q[2 * p + 1] = qb;
    }
  }
  if (lmax >= 0) atomicMax(&s_lmax, lmax);
  __syncthreads();
  const int l_hi = s_lmax;
  const int l_lo = (int)(m0.w & 255u);
  for (int l = l_hi; l >= l_lo; --l) {
#pragma unroll
    for (int u = 0; u < kMomPer; ++u) {
      const uint32_t p = (uint32_t)(u * kMomThreads + tid);
      if (p >= size) continue;
      const uint32_t w = s_word[p];
      if ((w >> 24) || (int)((w >> 16) & 255u) != l) continue;
      const uint32_t stop = w & 0xFFFFu;
      float M = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
      for (uint32_t k = p + 1; k < stop;) {
        const float4 mk = s_mom[k];
        const float dx = s_ox[k] + mk.x;
        const float dy = s_oy[k] + mk.y;
        const float dz = s_oz[k] + mk.z;
        M += mk.w;
        sx = fmaf(mk.w, dx, sx);
        sy = fmaf(mk.w, dy, sy);
        sz = fmaf(mk.w, dz, sz);
        const uint32_t s = s_word[k] & 0xFFFFu;
        k = s > k ? s : stop;
      }
      const float inv = M > 0.f ? 1.0f / M : 0.f;
      const float ox = sx * inv, oy = sy * inv, oz = sz * inv;
      s_mom[p] = make_float4(ox, oy, oz, M);
      if (QUAD) {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f;
        for (uint32_t k = p + 1; k < stop;) {
          const float4 mk = s_mom[k];
          const float4 qa = s_q[2 * k];
          const float4 qb = s_q[2 * k + 1];
          const float dx = s_ox[k] + mk.x - ox;
          const float dy = s_oy[k] + mk.y - oy;
          const float dz = s_oz[k] + mk.z - oz;
          const float wk = mk.w;
          s0 += qa.x + wk * dx * dx;
          s1 += qa.y + wk * dy * dy;
          s2 += qa.z + wk * dz * dz;
          s3 += qa.w + wk * dx * dy;
          s4 += qb.x + wk * dx * dz;
          s5 += qb.y + wk * dy * dz;
          const uint32_t s = s_word[k] & 0xFFFFu;
          k = s > k ? s : stop;
        }
        s_q[2 * p] = make_float4(s0, s1, s2, s3);
        s_q[2 * p + 1] = make_float4(s4, s5, 0.f, 0.f);
      }
    }
    __syncthreads();
  }
  // the root's terms in its parent's sums, for the top launch (a block's
  // root that is not a system's root has a top cell as parent)
  if (!QUAD && tid == 0 && (m0.w & 255u) != 0) {
    const uint32_t par = rec[c0].aux.x;
    const double4 gp = rec[par].geo;
    const int64_t k = 8 * (int64_t)rec[par].aux.y + cell_octant(wrec[c0]);
    const float4 mo = s_mom[0];
    if (k < slot_cap)
      slot[k] = make_float4((float)(gx[0] - gp.x) + mo.x,
                            (float)(gy[0] - gp.y) + mo.y,
                            (float)(gz[0] - gp.z) + mo.z, mo.w);
  }
#pragma unroll
  for (int u = 0; u < kMomPer; ++u) {
    const uint32_t p = (uint32_t)(u * kMomThreads + tid);
    if (p >= size) continue;
    const uint32_t c = c0 + p;
    const float4 mo = s_mom[p];
    mom[c] = mo;
    pm[c] = make_double4(gx[u] + (double)mo.x, gy[u] + (double)mo.y,
                         gz[u] + (double)mo.z, (double)mo.w);
    if (QUAD) {
      quad[2 * (int64_t)c] = s_q[2 * p];
      quad[2 * (int64_t)c + 1] = s_q[2 * p + 1];
    }
  }
}

// A top cell's sums from its children (ch: by octant, kNone where there is
// none), in pre-order as k_mom_internal takes them.  A child tagged
// kTopTag is a top cell: its moments are in LDS (s_mom, s_q) by top
// position when LDS, otherwise in global memory (its id from the top list).
template <bool QUAD, bool LDS>
__device__ __forceinline__ void top_sums(double gx, double gy, double gz,
                                         const uint32_t* ch,
                                         const uint32_t* __restrict__ top,
                                         const CellRec* __restrict__ rec,
                                         const float4* __restrict__ mom,
                                         const float4* __restrict__ quad,
                                         const float4* s_mom,
                                         const float4* s_q, float4& mo,
                                         float4& qa_out, float4& qb_out) {
  // per child: its moments, the FP32 offset of its centre from this cell's
  // (formed in FP64 and rounded once, as k_mom_internal forms it), and its
  // top position (kNone: not a top cell, or no LDS)
  float4 mk[8];
  float ex[8], ey[8], ez[8];
  uint32_t tp[8], kid[8];
  // kid: the child's cell id (a top child's from the top list; an absent
  // child reads cell 0 instead, so that its loads need no branch, and its
  // values are never used)
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const uint32_t e = ch[o];
    const bool tagged = e != kNone && (e & kTopTag);
    const uint32_t k = e == kNone ? 0u : (tagged ? top[e & ~kTopTag] : e);
    kid[o] = k;
    const double4 gk = rec[k].geo;
    mk[o] = mom[k];
    ex[o] = (float)(gk.x - gx);
    ey[o] = (float)(gk.y - gy);
    ez[o] = (float)(gk.z - gz);
    tp[o] = (LDS && tagged) ? (e & ~kTopTag) : kNone;
  }
  if (LDS) {
#pragma unroll
    for (int o = 0; o < 8; ++o)
      if (tp[o] != kNone) mk[o] = s_mom[tp[o]];
  }
  float M = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    if (ch[o] == kNone) continue;
    const float dx = ex[o] + mk[o].x;
    const float dy = ey[o] + mk[o].y;
    const float dz = ez[o] + mk[o].z;
    M += mk[o].w;
    sx = fmaf(mk[o].w, dx, sx);
    sy = fmaf(mk[o].w, dy, sy);
    sz = fmaf(mk[o].w, dz, sz);
  }
  const float inv = M > 0.f ? 1.0f / M : 0.f;
  const float ox = sx * inv, oy = sy * inv, oz = sz * inv;
  mo = make_float4(ox, oy, oz, M);
  if (!QUAD) return;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    if (ch[o] == kNone) continue;
    float4 qa, qb;
    if (LDS && tp[o] != kNone) {
      qa = s_q[2 * tp[o]];
      qb = s_q[2 * tp[o] + 1];
    } else {
      qa = quad[2 * (int64_t)kid[o]];
      qb = quad[2 * (int64_t)kid[o] + 1];
    }
    const float dx = ex[o] + mk[o].x - ox;
    const float dy = ey[o] + mk[o].y - oy;
    const float dz = ez[o] + mk[o].z - oz;
    const float w = mk[o].w;
    s0 += qa.x + w * dx * dx;
    s1 += qa.y + w * dy * dy;
    s2 += qa.z + w * dz * dz;
    s3 += qa.w + w * dx * dy;
    s4 += qb.x + w * dx * dz;
    s5 += qb.y + w * dy * dz;
  }
  qa_out = make_float4(s0, s1, s2, s3);
  qb_out = make_float4(s4, s5, 0.f, 0.f);
}

// The top cells, deepest level first, by one workgroup: a cell's children
// are blocks' roots (summed by the previous launch, read from global
// memory) or top cells one level deeper (summed before the last barrier by
// this workgroup).  Up to top_lds<QUAD>() top cells keep their centres,
// child tables and moments in LDS and are written out after the last
// barrier; beyond that the top cells go through global memory.
// Monopole moments of at most kMomTopThreads top cells (the common case):
// one per thread.  A child that is a block's root left its terms in the
// parent's slot (slot 8 j + octant: the FP32 centre offset plus COM offset,
// and the mass, as k_mom_internal forms them), so the loads before the
// level loop are contiguous per thread; a top child's centre and moments
// come from LDS by top position.  Only 40 KiB of LDS are allocated.
__global__ void __launch_bounds__(kMomTopThreads)
k_mom_top_one(const uint32_t* __restrict__ top,
              const uint32_t* __restrict__ tlo,
              const uint32_t* __restrict__ ctab,
              const float4* __restrict__ slot,
              const CellRec* __restrict__ rec, float4* __restrict__ mom,
              double4* __restrict__ pm) {
  __shared__ float4 s_mom[kMomTopThreads];
  __shared__ double s_gx[kMomTopThreads], s_gy[kMomTopThreads],
      s_gz[kMomTopThreads];
  const uint32_t n_top = tlo[kLevels];
  const uint32_t j = threadIdx.x;
  // a thread past the top cells works on the last one and writes nothing
  const uint32_t jj = j < n_top ? j : n_top - 1;
  const uint32_t c = top[jj];
  const double4 g = rec[c].geo;
  const int lv = j < n_top ? (int)(rec[c].meta.w & 255u) : -1;
  uint32_t ch[8];
  // per child: (dx, dy, dz, m) of a block root; (ex, ey, ez) of a top child
  float tx[8], ty[8], tz[8], tw[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    ch[o] = ctab[8 * (int64_t)jj + o];
    const float4 v = slot[8 * (int64_t)jj + o];
    tx[o] = v.x;
    ty[o] = v.y;
    tz[o] = v.z;
    tw[o] = v.w;
  }
  if (j < n_top) {
    s_gx[j] = g.x;
    s_gy[j] = g.y;
    s_gz[j] = g.z;
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const uint32_t e = ch[o];
    if (e != kNone && (e & kTopTag)) {
      const uint32_t tq = e & ~kTopTag;
      tx[o] = (float)(s_gx[tq] - g.x);
      ty[o] = (float)(s_gy[tq] - g.y);
      tz[o] = (float)(s_gz[tq] - g.z);
    }
  }
  for (int l = kLevels - 1; l >= 0; --l) {
    if (tlo[l] >= tlo[l + 1]) continue;  // uniform
    if (lv == l) {
      float M = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const uint32_t e = ch[o];
        if (e == kNone) continue;
        float dx = tx[o], dy = ty[o], dz = tz[o], w = tw[o];
        if (e & kTopTag) {
          const float4 m = s_mom[e & ~kTopTag];
          dx = tx[o] + m.x;
          dy = ty[o] + m.y;
          dz = tz[o] + m.z;
          w = m.w;
        }
        M += w;
        sx = fmaf(w, dx, sx);
        sy = fmaf(w, dy, sy);
        sz = fmaf(w, dz, sz);
      }
      const float inv = M > 0.f ? 1.0f / M : 0.f;
      s_mom[j] = make_float4(sx * inv, sy * inv, sz * inv, M);
    }
    __syncthreads();
  }
  if (j < n_top) {
    const float4 mo = s_mom[j];
    mom[c] = mo;
    pm[c] = make_double4(g.x + (double)mo.x, g.y + (double)mo.y,
                         g.z + (double)mo.z, (double)mo.w);
  }
}

template <bool QUAD>
constexpr int top_lds() { return QUAD ? kMomTopLds / 2 : kMomTopLds; }

template <bool QUAD>
__global__ void __launch_bounds__(kMomTopThreads)
k_mom_top(const uint32_t* __restrict__ top, const uint32_t* __restrict__ tlo,
          const uint32_t* __restrict__ ctab, const CellRec* __restrict__ rec,
          float4* __restrict__ mom, float4* __restrict__ quad,
          double4* __restrict__ pm) {
  constexpr int kCap = top_lds<QUAD>();
  __shared__ double s_gx[kCap], s_gy[kCap], s_gz[kCap];
  __shared__ float4 s_mom[kCap];
  __shared__ uint32_t s_ch[8 * kCap];
  __shared__ float4 s_q[QUAD ? 2 * kCap : 1];
  const uint32_t n_top = tlo[kLevels];
  if (n_top <= (uint32_t)kCap) {
    for (uint32_t i = threadIdx.x; i < 8 * n_top; i += kMomTopThreads)
      s_ch[i] = ctab[i];
    constexpr int kPer = (kCap + kMomTopThreads - 1) / kMomTopThreads;
    int lv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const uint32_t j = threadIdx.x + (uint32_t)(u * kMomTopThreads);
      lv[u] = -1;
      if (j >= n_top) continue;
      const uint32_t c = top[j];
      const double4 g = rec[c].geo;
      lv[u] = (int)(rec[c].meta.w & 255u);
      s_gx[j] = g.x;
      s_gy[j] = g.y;
      s_gz[j] = g.z;
    }
    __syncthreads();
    for (int l = kLevels - 1; l >= 0; --l) {
      if (tlo[l] >= tlo[l + 1]) continue;  // uniform
#pragma unroll 1
      for (int u = 0; u < kPer; ++u) {
        if (lv[u] != l) continue;
        const uint32_t j = threadIdx.x + (uint32_t)(u * kMomTopThreads);
        uint32_t ch[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) ch[o] = s_ch[8 * j + o];
        float4 mo, qa, qb;
        top_sums<QUAD, true>(s_gx[j], s_gy[j], s_gz[j], ch, top, rec, mom,
                             quad, s_mom, s_q, mo, qa, qb);
        s_mom[j] = mo;
        if (QUAD) {
          s_q[2 * j] = qa;
          s_q[2 * j + 1] = qb;
        }
      }
      __syncthreads();
    }
    for (uint32_t j = threadIdx.x; j < n_top; j += kMomTopThreads) {
      const uint32_t c = top[j];
      const float4 mo = s_mom[j];
      mom[c] = mo;
      pm[c] = make_double4(s_gx[j] + (double)mo.x, s_gy[j] + (double)mo.y,
                           s_gz[j] + (double)mo.z, (double)mo.w);
      if (QUAD) {
        quad[2 * (int64_t)c] = s_q[2 * j];
        quad[2 * (int64_t)c + 1] = s_q[2 * j + 1];
      }
    }
    return;
  }
  for (int l = kLevels - 1; l >= 0; --l) {
    const uint32_t a = tlo[l], b = tlo[l + 1];
    if (a >= b) continue;  // uniform
    for (uint32_t j = a + threadIdx.x; j < b; j += kMomTopThreads) {
      const uint32_t c = top[j];
      const double4 g = rec[c].geo;
      uint32_t ch[8];
#pragma unroll
      for (int o = 0; o < 8; ++o) ch[o] = ctab[8 * (int64_t)j + o];
      float4 mo, qa, qb;
      top_sums<QUAD, false>(g.x, g.y, g.z, ch, top, rec, mom, quad, nullptr,
                            nullptr, mo, qa, qb);
      mom[c] = mo;
      pm[c] = make_double4(g.x + (double)mo.x, g.y + (double)mo.y,
                           g.z + (double)mo.z, (double)mo.w);
      if (QUAD) {
        quad[2 * (int64_t)c] = qa;
        quad[2 * (int64_t)c + 1] = qb;
      }
    }
    __syncthreads();
  }
}
}  // namespace

// The chunk table (system, first, end) of the bounding-box pass is built on
// the host whenever the particles or the systems change.
int launch_root(nb_ctx* c) {
  const size_t nch = c->h_bbox_chunks.size();
  int rc = reserve(c, c->bbox_part, nch * 8);
  if (!rc) rc = reserve(c, c->root, (size_t)c->n_sys);
  if (rc) return rc;
  hipLaunchKernelGGL(k_bbox_partial, dim3((unsigned)nch), dim3(kBboxThreads),
                     0, c->stream, (const double4*)c->pos.p,
                     (const int4*)c->bbox_chunks.p, c->bbox_part.p);
  const double r1 = 1.0 / c->cfg.theta;
  const double rr = r1 * r1;
  hipLaunchKernelGGL(k_bbox_final, dim3((unsigned)c->n_sys),
                     dim3(kBboxThreads), 0, c->stream,
                     (const double*)c->bbox_part.p,
                     (const uint32_t*)c->bbox_first.p, rr, c->root.p);
  if (c->n_sys > 1)
    hipLaunchKernelGGL(k_bbox_bad, dim3(1), dim3(64), 0, c->stream, c->root.p,
                       c->n_sys);
  return hip_check(c, hipGetLastError(), "root launch");
}

int launch_keys(nb_ctx* c) {
  int rc = reserve(c, c->key, (size_t)c->n);
  if (!rc) rc = reserve(c, c->val, (size_t)c->n);
  if (rc) return rc;
  hipLaunchKernelGGL(k_keys, dim3(grid_for(c->n, 256)), dim3(256), 0,
                     c->stream, (const double4*)c->pos.p, c->n,
                     (const Root*)c->root.p, (const uint32_t*)c->seg.p,
                     c->key.p);
  return hip_check(c, hipGetLastError(), "keys launch");
}

// Upload the system offsets and the bounding-box chunk table, and fill the
// per-slot system ids.  Called by nb_set_particles / nb_set_systems.
int launch_seg_fill(nb_ctx* c) {
  constexpr int64_t kChunk = 16384;
  std::vector<uint32_t> off(c->n_sys + 1), first(c->n_sys + 1);
  c->h_bbox_chunks.clear();
  for (int64_t s = 0; s < c->n_sys; ++s) {
    off[s] = (uint32_t)c->h_sys_off[s];
    first[s] = (uint32_t)c->h_bbox_chunks.size();
    for (int64_t b = c->h_sys_off[s]; b < c->h_sys_off[s + 1]; b += kChunk) {
      const int64_t e = std::min(b + kChunk, c->h_sys_off[s + 1]);
      c->h_bbox_chunks.push_back(make_int4((int)s, (int)b, (int)e, 0));
    }
  }
  off[c->n_sys] = (uint32_t)c->n;
  first[c->n_sys] = (uint32_t)c->h_bbox_chunks.size();
  int rc = reserve(c, c->sys_off, off.size());
  if (!rc) rc = reserve(c, c->bbox_first, first.size());
  if (!rc) rc = reserve(c, c->bbox_chunks, c->h_bbox_chunks.size());
  if (!rc) rc = reserve(c, c->seg, (size_t)c->n);
  if (!rc) rc = reserve(c, c->croot, (size_t)c->n_sys + 1);
  if (rc) return rc;
  rc = hip_check(c, hipMemcpy(c->sys_off.p, off.data(), off.size() * 4,
                              hipMemcpyHostToDevice), "system upload");
  if (!rc) rc = hip_check(c, hipMemcpy(c->bbox_first.p, first.data(),
                                       first.size() * 4,
                                       hipMemcpyHostToDevice), "system upload");
  if (!rc) rc = hip_check(c, hipMemcpy(c->bbox_chunks.p,
                                       c->h_bbox_chunks.data(),
                                       c->h_bbox_chunks.size() * sizeof(int4),
                                       hipMemcpyHostToDevice), "system upload");
  if (rc) return rc;
  hipLaunchKernelGGL(k_seg_fill, dim3(grid_for(c->n, 256)), dim3(256), 0,
                     c->stream, (const uint32_t*)c->sys_off.p, c->n_sys, c->n,
                     c->seg.p);
  return hip_check(c, hipGetLastError(), "system fill launch");
}

int launch_reorder(nb_ctx* c) {
  const size_t n = (size_t)c->n;
  int rc = reserve(c, c->pos2, n);
  if (!rc) rc = reserve(c, c->vx2, n);
  if (!rc) rc = reserve(c, c->vy2, n);
  if (!rc) rc = reserve(c, c->vz2, n);
  if (!rc) rc = reserve(c, c->orig2, n);
  if (rc) return rc;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(c->n, 256)), dim3(256), 0,
                     c->stream, c->n, (const uint32_t*)c->val.p,
                     (const double4*)c->pos.p, (const double*)c->vx.p,
                     (const double*)c->vy.p, (const double*)c->vz.p,
                     (const uint32_t*)c->orig.p, c->pos2.p, c->vx2.p,
                     c->vy2.p, c->vz2.p, c->orig2.p);
  std::swap(c->pos, c->pos2);
  std::swap(c->vx, c->vx2);
  std::swap(c->vy, c->vy2);
  std::swap(c->vz, c->vz2);
  std::swap(c->orig, c->orig2);
  return hip_check(c, hipGetLastError(), "reorder launch");
}

int launch_link_count(nb_ctx* c) {
  const size_t n = (size_t)c->n;
  int rc = reserve(c, c->lam, n);
  if (!rc) rc = reserve(c, c->lmin, n);
  if (!rc) rc = reserve(c, c->cstart, n + 1);
  if (rc) return rc;
  hipLaunchKernelGGL(k_link_count, dim3(grid_for(c->n, 256)), dim3(256), 0,
                     c->stream, (const uint64_t*)c->key.p, c->n,
                     (int)c->cfg.n_leaf, (const uint32_t*)c->seg.p,
                     (const uint32_t*)c->sys_off.p, c->lam.p, c->lmin.p,
                     c->cstart.p);
  rc = hip_check(c, hipGetLastError(), "link count launch");
  if (rc) return rc;
  return scan_u32(c, c->cstart.p, c->cstart.p, c->n);
}

int launch_link_fill(nb_ctx* c) {
  int rc = reserve(c, c->c_rec, (size_t)c->n_cell);
  if (!rc) rc = reserve(c, c->c_wrec, (size_t)c->n_cell);
  if (rc) return rc;
  hipLaunchKernelGGL(k_link_fill, dim3(grid_for(c->n, 256)), dim3(256), 0,
                     c->stream, (const uint64_t*)c->key.p, c->n,
                     (const uint32_t*)c->seg.p, (const uint32_t*)c->sys_off.p,
                     (const uint8_t*)c->lam.p, (const uint8_t*)c->lmin.p,
                     (const uint32_t*)c->cstart.p, (const Root*)c->root.p,
                     c->c_rec.p, c->c_wrec.p);
  hipLaunchKernelGGL(k_sys_roots, dim3(grid_for(c->n_sys + 1, 256)),
                     dim3(256), 0, c->stream, (const uint32_t*)c->cstart.p,
                     (const uint32_t*)c->sys_off.p, c->n_sys, c->croot.p);
  return hip_check(c, hipGetLastError(), "link fill launch");
}

// Group flags and their scan.
int launch_group_flags(nb_ctx* c) {
  int rc = reserve(c, c->gflag, (size_t)c->n_cell + 1);
  if (rc) return rc;
  hipLaunchKernelGGL(k_group_flags, dim3(grid_for(c->n_cell, 256)), dim3(256),
                     0, c->stream, c->n_cell, (const CellRec*)c->c_rec.p,
                     (int)c->cfg.n_grp, c->gflag.p);
  rc = hip_check(c, hipGetLastError(), "group flags launch");
  if (rc) return rc;
  return scan_u32(c, c->gflag.p, c->gflag.p, c->n_cell);
}

// Level lists by counting sort; also stages the bucket starts and the group
// count in c->lvl_stage for the host to read.
int launch_level_lists(nb_ctx* c) {
  const int nblk = (int)grid_for(c->n_cell, kBkTile);
  int rc = reserve(c, c->lvl_cells, (size_t)c->n_cell);
  if (!rc) rc = reserve(c, c->bucket, (size_t)kBuckets * nblk + 1);
  if (!rc) rc = reserve(c, c->lvl_stage, kLevels + 4);
  if (rc) return rc;
  hipLaunchKernelGGL(k_bucket_hist, dim3(nblk), dim3(kBkThreads), 0,
                     c->stream, c->n_cell, (const CellRec*)c->c_rec.p,
                     c->bucket.p, nblk);
  rc = hip_check(c, hipGetLastError(), "bucket launch");
  if (rc) return rc;
  rc = scan_u32(c, c->bucket.p, c->bucket.p, (int64_t)kBuckets * nblk);
  if (rc) return rc;
  hipLaunchKernelGGL(k_bucket_scatter, dim3(nblk), dim3(kBkThreads), 0,
                     c->stream, c->n_cell, (const CellRec*)c->c_rec.p,
                     (const uint32_t*)c->bucket.p, nblk, c->lvl_cells.p);
  hipLaunchKernelGGL(k_bucket_starts, dim3(1), dim3(64), 0, c->stream,
                     (const uint32_t*)c->bucket.p, nblk,
                     (const uint32_t*)c->gflag.p, c->n_cell,
                     c->lvl_stage.p);
  return hip_check(c, hipGetLastError(), "bucket scatter launch");
}

// Blocks and top cells of the moment pass (the tree's topology is fixed
// until the next construction).  Top cells at one level have disjoint
// subtrees of more than kMomBlock cells, so there are at most
// kLevels n_cell / (kMomBlock + 1) of them.
int launch_mom_plan(nb_ctx* c) {
  const int64_t nc = c->n_cell;
  const int64_t top_cap = kLevels * nc / (kMomBlock + 1) + 1;
  int rc = reserve(c, c->mp_bflag, (size_t)nc + 1);
  if (!rc) rc = reserve(c, c->mp_tflag, (size_t)nc + 1);
  if (!rc) rc = reserve(c, c->mp_blocks, (size_t)nc);
  if (!rc) rc = reserve(c, c->mp_top, (size_t)top_cap);
  if (!rc) rc = reserve(c, c->mp_tlo, kLevels + 1);
  if (!rc) rc = reserve(c, c->mp_ctab, 8 * (size_t)top_cap);
  if (!rc) rc = reserve(c, c->mp_slot, 8 * (size_t)top_cap);
  c->mp_slot_cap = 8 * top_cap;
  if (rc) return rc;
  const unsigned grid = grid_for(nc, 256);
  hipLaunchKernelGGL(k_mp_flags, dim3(grid), dim3(256), 0, c->stream, nc,
                     (const CellRec*)c->c_rec.p, c->mp_bflag.p);
  rc = hip_check(c, hipGetLastError(), "block flags launch");
  if (!rc) rc = scan_u32(c, c->mp_bflag.p, c->mp_bflag.p, nc);
  if (rc) return rc;
  hipLaunchKernelGGL(k_mp_blocks, dim3(grid), dim3(256), 0, c->stream, nc,
                     (const uint32_t*)c->mp_bflag.p, c->mp_blocks.p);
  hipLaunchKernelGGL(k_mp_tflags, dim3(grid), dim3(256), 0, c->stream, nc,
                     (const uint32_t*)c->lvl_cells.p,
                     (const CellRec*)c->c_rec.p, c->mp_tflag.p);
  rc = hip_check(c, hipGetLastError(), "top flags launch");
  if (!rc) rc = scan_u32(c, c->mp_tflag.p, c->mp_tflag.p, nc);
  if (rc) return rc;
  hipLaunchKernelGGL(k_mp_top, dim3(grid), dim3(256), 0, c->stream, nc,
                     (const uint32_t*)c->lvl_cells.p,
                     (const uint32_t*)c->mp_tflag.p, c->mp_top.p, top_cap,
                     c->c_rec.p);
  const int64_t ctab_cap = 8 * top_cap;
  hipLaunchKernelGGL(k_mp_tlo, dim3(grid_for(ctab_cap, 256)), dim3(256), 0,
                     c->stream, nc, (const uint32_t*)c->lvl_stage.p,
                     (const uint32_t*)c->mp_tflag.p,
                     (const uint32_t*)c->mp_bflag.p, c->mp_tlo.p,
                     c->lvl_stage.p + kLevels + 2, c->mp_ctab.p, top_cap);
  hipLaunchKernelGGL(k_mp_ctab, dim3(grid), dim3(256), 0, c->stream, nc,
                     (const CellRec*)c->c_rec.p, (const uint4*)c->c_wrec.p,
                     c->mp_ctab.p, ctab_cap);
  return hip_check(c, hipGetLastError(), "moment plan launch");
}

int launch_moments(nb_ctx* c) {
  const size_t nc = (size_t)c->n_cell;
  int rc = reserve(c, c->c_mom, nc);
  if (!rc) rc = reserve(c, c->c_pm, nc);
  if (!rc) rc = reserve(c, c->c_quad, 2 * nc);
  if (rc) return rc;
  const bool quad = c->cfg.order == 2;
  if (!(c->cfg.flags & NB_FLAG_LEVEL_MOMENTS)) {
    // two launches: the blocks (leaves included), then the top cells
    if (c->mp_nblk > 0) {
      auto blk = quad ? k_mom_block<true> : k_mom_block<false>;
      hipLaunchKernelGGL(blk, dim3((unsigned)c->mp_nblk), dim3(kMomThreads),
                         0, c->stream, (const uint32_t*)c->mp_blocks.p,
                         (const CellRec*)c->c_rec.p, (const uint4*)c->c_wrec.p,
                         (const double4*)c->pos.p, c->c_mom.p, c->c_quad.p,
                         c->c_pm.p, c->mp_slot.p, c->mp_slot_cap);
    }
    if (c->mp_ntop > 0 && !quad && c->mp_ntop <= kMomTopThreads) {
      hipLaunchKernelGGL(k_mom_top_one, dim3(1), dim3(kMomTopThreads), 0,
                         c->stream, (const uint32_t*)c->mp_top.p,
                         (const uint32_t*)c->mp_tlo.p,
                         (const uint32_t*)c->mp_ctab.p,
                         (const float4*)c->mp_slot.p,
                         (const CellRec*)c->c_rec.p, c->c_mom.p, c->c_pm.p);
    } else if (c->mp_ntop > 0) {
      auto top = quad ? k_mom_top<true> : k_mom_top<false>;
      hipLaunchKernelGGL(top, dim3(1), dim3(kMomTopThreads), 0, c->stream,
                         (const uint32_t*)c->mp_top.p,
                         (const uint32_t*)c->mp_tlo.p,
                         (const uint32_t*)c->mp_ctab.p,
                         (const CellRec*)c->c_rec.p, c->c_mom.p, c->c_quad.p,
                         c->c_pm.p);
    }
  } else {
    // one launch per level (leaves, then the internal levels bottom-up)
    auto leaf = quad ? k_mom_leaf<true> : k_mom_leaf<false>;
    auto inner = quad ? k_mom_internal<true> : k_mom_internal<false>;
    if (c->n_leaves > 0)
      hipLaunchKernelGGL(leaf, dim3(grid_for(kLeafLanes * c->n_leaves, 256)),
                         dim3(256), 0,
                         c->stream, c->n_leaves,
                         (const uint32_t*)c->lvl_cells.p + c->lvl_off[kLevels],
                         (const CellRec*)c->c_rec.p, (const double4*)c->pos.p,
                         c->c_mom.p, c->c_quad.p, c->c_pm.p);
    for (int l = kMaxLevel - 1; l >= 0; --l) {
      const int64_t cnt = c->lvl_count[l];
      if (cnt == 0) continue;
      hipLaunchKernelGGL(inner, dim3(grid_for(cnt, 256)), dim3(256), 0,
                         c->stream, cnt,
                         (const uint32_t*)c->lvl_cells.p + c->lvl_off[l],
                         (const CellRec*)c->c_rec.p, c->c_mom.p, c->c_quad.p,
                         c->c_pm.p);
    }
  }
  rc = hip_check(c, hipGetLastError(), "moments launch");
  if (!rc && c->learn) rc = launch_com(c);
  return rc;
}

// Tight boxes of every group's particles at the current positions.
int launch_group_box(nb_ctx* c, double4* lo, double4* hi) {
  hipLaunchKernelGGL(k_group_box, dim3(grid_for(c->n_groups, 4)), dim3(256),
                     0, c->stream, c->n_groups, (const uint32_t*)c->g_begin.p,
                     (const uint32_t*)c->g_count.p, (const double4*)c->pos.p,
                     lo, hi);
  return hip_check(c, hipGetLastError(), "group box launch");
}

// How to split the last n < 64 particles of a group into work items.  A
// chunk of s particles runs on r = 64 / s lane slices, so a list entry
// costs about 14 / r vector instructions plus a fixed share for staging it
// in LDS; the split minimises the sum (dynamic programming over n).  For
// example 40 -> 8 + 32, 33 -> 1 + 32, 63 -> 63.
static ChunkTable chunk_table() {
  ChunkTable t;
  const double stage = 0.5;
  double best[64];
  int pick[64];
  best[0] = 0.0;
  pick[0] = 0;
  for (int n = 1; n < 64; ++n) {
    best[n] = 1e30;
    pick[n] = n;
    for (int s = 1; s <= n; ++s) {
      const double cst = 14.0 / (64 / s) + stage + best[n - s];
      if (cst < best[n] - 1e-12) {
        best[n] = cst;
        pick[n] = s;
      }
    }
  }
  t.e[0] = 0;
  for (int n = 1; n < 64; ++n) {
    uint32_t e = 0, cnt = 0;
    int r = n;
    for (; r > 0 && cnt < 3; r -= pick[r]) e |= (uint32_t)pick[r] << (8 * cnt++);
    // the chunks must cover all n particles; otherwise keep one chunk
    t.e[n] = r == 0 ? (e | cnt << 24) : ((uint32_t)n | 1u << 24);
  }
  return t;
}

int launch_group_fill(nb_ctx* c) {
  static const ChunkTable tab = chunk_table();
  const size_t ng = (size_t)c->n_groups;
  int rc = reserve(c, c->g_cell, ng);
  if (!rc) rc = reserve(c, c->g_begin, ng);
  if (!rc) rc = reserve(c, c->g_count, ng);
  if (!rc) rc = reserve(c, c->g_lo, ng);
  if (!rc) rc = reserve(c, c->g_hi, ng);
  if (!rc) rc = reserve(c, c->g_chunks, ng + 1);
  if (!rc) rc = reserve(c, c->wi, 3 * ng + (size_t)c->n / 64 + 1);
  if (rc) return rc;
  hipLaunchKernelGGL(k_group_fill, dim3(grid_for(c->n_cell, 256)), dim3(256),
                     0, c->stream, c->n_cell, (const uint32_t*)c->gflag.p,
                     (const CellRec*)c->c_rec.p, tab, c->g_cell.p,
                     c->g_begin.p, c->g_count.p, c->g_chunks.p);
  rc = launch_group_box(c, c->g_lo.p, c->g_hi.p);
  if (rc) return rc;
  rc = scan_u32(c, c->g_chunks.p, c->g_chunks.p, c->n_groups);
  if (rc) return rc;
  hipLaunchKernelGGL(k_make_wi, dim3(grid_for(c->n_groups, 256)), dim3(256),
                     0, c->stream, c->n_groups, (const uint32_t*)c->g_begin.p,
                     (const uint32_t*)c->g_count.p, tab,
                     (const uint32_t*)c->g_chunks.p, c->wi.p);
  return hip_check(c, hipGetLastError(), "work item launch");
}

}  // namespace nb
