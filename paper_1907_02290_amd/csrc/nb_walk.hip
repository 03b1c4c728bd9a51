// nb_walk.hip -- group-wise tree walk emitting index interaction lists
// (section 4.3 list construction; indirect addressing of section 4.1: the
// lists hold 32-bit indices, particles by internal slot, superparticles by
// cell id).
//
// The walk of one group is a stackless DFS over the pre-order cell array,
// jumping over a subtree with its skip id, run by a tile of lanes (few
// groups) or cut into stretches walked by kSplitLanes lanes (many groups,
// and refresh mode).  The opening test compares the
// squared distance from the group's tight box to the cell's geometric centre
// with (side / theta)^2 in FP64, evaluated term by term (no fused
// multiply-add: this file is built with -ffp-contract=off and uses explicit
// rounding intrinsics), so that lists are bit-identical to an FP64 reference.
// A cell whose particle range holds the group is always opened.
//
// Count pass, exclusive scans, fill pass: no atomics, ids in ascending
// order.  The fill pass writes one token per accepted cell (SPJ) or opened
// leaf, in walk order, staged per lane in LDS and written out in aligned
// 64-byte segments; a second kernel, one wave per group, splits the tokens
// into the SPJ list and the particle ids (EPJ) of the opened leaves, with
// whole wavefronts writing contiguous stretches.
// Workgroups are remapped so that each XCD walks a contiguous stretch of
// groups (Morton order), whose tree paths share that XCD's L2.
#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kWalkThreads = 256;
// Walk layout.  From kThreadWalkFrom groups on, kSplitLanes lanes per group,
// each walking one stretch of the pre-order array (k_walk_c); below, tiles
// of at least kTileWalk lanes, widened until about kTileLanes lanes are in
// flight (1.8k groups of a 2^22-particle disk: 0.5 ms in tiles against
// 2.4 ms one thread per group).  Refresh mode walks kSplitLanes lanes per
// group at every size (k_walk_r).
constexpr int64_t kThreadWalkFrom = 8192;
constexpr int kTileWalk = 4;
constexpr int64_t kTileLanes = 1 << 18;

__device__ inline int64_t xcd_block(int64_t nblk) {
  const int64_t per = (nblk + 7) / 8;
  return (int64_t)(blockIdx.x & 7u) * per + (int64_t)(blockIdx.x >> 3);
}

// Blocks that hold work when only the first *n_dev of n_walk items (`per`
// items per block) are to be walked: the XCD stretches are cut over those
// blocks, not over the launch's (sized for n_walk), so the work spreads
// over every XCD.
__device__ inline int64_t active_blocks(int64_t nblk, int64_t n_walk,
                                        const uint32_t* n_dev, int64_t per) {
  if (!n_dev) return nblk;
  const int64_t n = (int64_t)*n_dev < n_walk ? (int64_t)*n_dev : n_walk;
  return (n + per - 1) / per;
}

// Tokens of the fill pass: an accepted cell (SPJ) is its id, an opened
// leaf is its id with the top bit set.
constexpr uint32_t kLeafTag = 0x80000000u;
constexpr int kSeg = 16;  // tokens per 64-byte output segment
constexpr int kExpandBatch = 4;  // 64-token chunks per round of k_expand

// The walk over the 16-byte walk records (one load per visit instead of the
// 64-byte cell record's three), S lanes per group (S = 2, 4 or 8).  The
// stackless walk reaches the deepest cell gd holding the group, and every
// ancestor a of gd holds the group and is opened, so the walk visits a and
// skip(a) (the first cell after a's subtree, whose ancestors are ancestors of
// a).  Those cells cut the pre-order walk into S independent stretches: with
// a_1 .. a_{S/2-1} the ancestors of gd at depths D q / (S / 2) (D = depth of
// gd), lane h < S/2 walks the cells from a_h to a_{h+1} (a_0 = the system's
// root, a_{S/2} = gd) and lane S/2 + h the cells from skip(a_{S/2-h}) to
// skip(a_{S/2-h-1}) (skip(a_{S/2}) read as gd, skip(a_0) as the system's
// end), and the lanes' tokens in lane order are the one-thread walk's.  A
// terminal cell inside a stretch never reaches past its end: a subtree that
// held the stretch's end would hold an ancestor of the group and be opened.
// On the 2^20 disk (seeded sample of groups) the longest stretch of a group
// averages 1678 visits with two lanes and 843 with eight.  In slab mode each
// lane has a slab of its own (group g: slabs S g .. S g + S - 1); in the
// exact fill lane h writes after the tokens that the count pass recorded
// for lanes 0 .. h - 1 (cnt_tl, S per group).  The centre and
// (side / theta)^2 of a cell come from its integer coordinates and level by
// the tree build's own FP64 operations, so every opening decision, and the
// token stream, is the same as from the cell records.  A cell holds the
// group's particle range exactly when it is an ancestor of, or is, the
// deepest cell with that range (cell ranges are nested or disjoint and never
// empty), i.e. when c <= gd < skip(c) in pre-order.
template <bool FILL, int S>
__global__ void __launch_bounds__(kWalkThreads)
k_walk_c(int64_t n_walk, int64_t nblk, const uint32_t* __restrict__ g_begin,
         const uint32_t* __restrict__ g_count,
         const double4* __restrict__ g_lo, const double4* __restrict__ g_hi,
         const uint32_t* __restrict__ g_cell, const CellRec* __restrict__ rec,
         const uint4* __restrict__ wrec, const Root* __restrict__ roots,
         const uint32_t* __restrict__ seg, const uint32_t* __restrict__ croot,
         uint32_t* __restrict__ cnt_e, uint32_t* __restrict__ cnt_s,
         uint32_t* __restrict__ cnt_t, uint32_t* __restrict__ cnt_tl,
         const uint64_t* __restrict__ tok_off,
         uint32_t* __restrict__ tok, uint32_t slab) {
  static_assert(S == 2 || S == 4 || S == 8, "lanes per group");
  constexpr int H = S / 2;
  __shared__ uint32_t stage[FILL ? kSeg : 1][kWalkThreads];
  const int64_t blk = xcd_block(nblk);
  if (blk >= nblk) return;
  // n_walk = S x groups: the S lanes of a group leave together
  const int64_t tt = blk * kWalkThreads + threadIdx.x;
  if (tt >= n_walk) return;
  const int64_t g = tt / S;
  const int h = (int)(tt % S);
  const uint32_t gb = g_begin[g];
  const uint32_t ge = gb + g_count[g];
  const double4 lo = g_lo[g], hi = g_hi[g];
  // deepest cell whose range is the group's: down the chain of only children
  uint32_t gd = g_cell[g];
  for (;;) {
    if ((rec[gd].meta.w >> 8) & 1u) break;
    const uint4 m1 = rec[gd + 1].meta;
    if (m1.x != gb || m1.y != ge) break;
    ++gd;
  }
  const uint32_t sys = seg[gb];
  const uint32_t r0 = croot[sys], r1 = croot[sys + 1];
  // this lane's stretch [c, nc)
  uint32_t c, nc;
  if (S == 2) {
    c = h ? gd : r0;
    nc = h ? r1 : gd;
  } else {
    // ancestors of gd at depths D q / H, q = 1 .. H - 1 (one cell per level
    // on the path: the parent of a level-l cell is at level l - 1)
    const int D = (int)(rec[gd].meta.w & 255u);
    uint32_t a[H + 1];
    a[0] = r0;
    a[H] = gd;
    uint32_t x = gd;
    int lx = D;
#pragma unroll
    for (int q = H - 1; q >= 1; --q) {
      const int want = (D * q) / H;
      while (lx > want) {
        x = rec[x].aux.x;
        --lx;
      }
      a[q] = x;
    }
    if (h < H) {
      c = a[h];
      nc = a[h + 1];
    } else {
      const int k2 = h - H;  // 0 .. H - 1
      c = k2 == 0 ? gd : wrec[a[H - k2]].z;
      nc = k2 == H - 1 ? r1 : wrec[a[H - 1 - k2]].z;
    }
  }
  uint32_t* dst = nullptr;
  uint64_t out = 0;
  uint64_t end = 0;
  int sc = 0;
  if (FILL) {
    if (slab) {
      out = ((uint64_t)g * S + (uint64_t)h) * slab;
      end = out + slab;
    } else {
      out = tok_off[g];
      for (int q = 0; q < h; ++q) out += cnt_tl[(uint64_t)g * S + q];
      end = ~0ull;
    }
    dst = tok;
  }
  const bool counts = !FILL || slab != 0;
  uint32_t ne = 0, ns = 0, nl = 0;
  const Root* root = roots + sys;
  const double rx = root->lo[0], ry = root->lo[1], rz = root->lo[2];
  const double rr = root->rr;
  const int k = root->k;
  // Loads and stores share one completion counter, so the wait for a
  // visit's record also waits for every store issued before it.  A full
  // segment read from the stage is therefore stored in the next visit, right
  // after that visit's record has arrived: the stores then have a whole
  // visit to complete before the following wait.  The loop-invariant loads
  // are completed before the loop, so that its head needs no wait.
  asm volatile("" ::"v"(c), "v"(nc), "v"(gd), "v"(k), "v"(rr), "v"(rx),
               "v"(ry), "v"(rz));
  asm volatile("" ::"v"(lo.x), "v"(lo.y), "v"(lo.z), "v"(hi.x), "v"(hi.y),
               "v"(hi.z), "v"(gb));
  uint4 seg0, seg1, seg2, seg3;
  uint32_t* pend = nullptr;
  while (c < nc) {
    const uint4 w = wrec[c];
    // all four words in registers here: otherwise the compiler loads the
    // coordinates separately inside the opening test, a second round trip
    // to memory after the first
    asm volatile("" ::"v"(w.x), "v"(w.y), "v"(w.z), "v"(w.w));
    if (FILL && pend) {
      uint4* d4 = reinterpret_cast<uint4*>(pend);
      d4[0] = seg0;
      d4[1] = seg1;
      d4[2] = seg2;
      d4[3] = seg3;
      pend = nullptr;
    }
    const uint32_t skip = w.z;
    const bool leaf = (w.y >> 31) != 0u;
    // the opening test for every cell (branch-free: with about one wave per
    // SIMD each divergent branch costs its full latency)
    const int l = (int)(w.w & 31u);
    const uint64_t q = (uint64_t)w.x | ((uint64_t)(w.y & 0x7FFFFFFFu) << 32);
    const uint32_t qx = (uint32_t)q & 0x1FFFFFu;
    const uint32_t qy = (uint32_t)(q >> 21) & 0x1FFFFFu;
    const uint32_t qz = (uint32_t)(q >> 42);
    const double half = ldexp(1.0, k - l - 1);
    const double cx = __dadd_rn(rx, __dmul_rn((double)(2u * qx + 1u), half));
    const double cy = __dadd_rn(ry, __dmul_rn((double)(2u * qy + 1u), half));
    const double cz = __dadd_rn(rz, __dmul_rn((double)(2u * qz + 1u), half));
    const double dx = fmax(fmax(__dsub_rn(lo.x, cx), __dsub_rn(cx, hi.x)), 0.0);
    const double dy = fmax(fmax(__dsub_rn(lo.y, cy), __dsub_rn(cy, hi.y)), 0.0);
    const double dz = fmax(fmax(__dsub_rn(lo.z, cz), __dsub_rn(cz, hi.z)), 0.0);
    const double d2 =
        __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                  __dmul_rn(dz, dz));
    // a cell holding the group is opened whatever its distance
    const bool open = (c <= gd && gd < skip) || !(d2 > ldexp(rr, 2 * (k - l)));
    const bool term = !open || leaf;   // accepted, or an opened leaf
    const uint32_t next = term ? skip : c + 1;
    if (next <= c) break;
    ns += open ? 0u : 1u;
    uint32_t cnt = w.w >> 5;
    if (cnt == kWalkCountSat) cnt = rec[c].meta.y - rec[c].meta.x;
    const bool opened_leaf = open && leaf;
    nl += opened_leaf ? 1u : 0u;
    ne += opened_leaf ? cnt : 0u;
    if (FILL) {
      // slot sc is free: write it every visit, keep it only for a token
      stage[sc][threadIdx.x] = open ? (c | kLeafTag) : c;
      sc += term ? 1 : 0;
      if (term && ((out + sc) & (kSeg - 1)) == 0) {
        if (out + sc > end) {
          // past the slab: drop
        } else if (sc == kSeg) {
          seg0 = make_uint4(stage[0][threadIdx.x], stage[1][threadIdx.x],
                            stage[2][threadIdx.x], stage[3][threadIdx.x]);
          seg1 = make_uint4(stage[4][threadIdx.x], stage[5][threadIdx.x],
                            stage[6][threadIdx.x], stage[7][threadIdx.x]);
          seg2 = make_uint4(stage[8][threadIdx.x], stage[9][threadIdx.x],
                            stage[10][threadIdx.x], stage[11][threadIdx.x]);
          seg3 = make_uint4(stage[12][threadIdx.x], stage[13][threadIdx.x],
                            stage[14][threadIdx.x], stage[15][threadIdx.x]);
          pend = dst + out;
        } else {
          for (int r = 0; r < sc; ++r) dst[out + r] = stage[r][threadIdx.x];
        }
        out += sc;
        sc = 0;
      }
    }
    c = next;
  }
  if (FILL && pend) {
    uint4* d4 = reinterpret_cast<uint4*>(pend);
    d4[0] = seg0;
    d4[1] = seg1;
    d4[2] = seg2;
    d4[3] = seg3;
  }
  if (FILL && out + sc <= end) {
    for (int q = 0; q < sc; ++q) dst[out + q] = stage[q][threadIdx.x];
  }
  if (counts) {
    const uint32_t ta = ns + nl;
    uint32_t e2 = ne, s2 = ns, t2 = ta;
#pragma unroll
    for (int o = S / 2; o > 0; o >>= 1) {
      e2 += __shfl_xor(e2, o, 64);
      s2 += __shfl_xor(s2, o, 64);
      t2 += __shfl_xor(t2, o, 64);
    }
    cnt_tl[(uint64_t)g * S + h] = ta;
    if (h == 0) {
      cnt_e[g] = e2;
      cnt_s[g] = s2;
      cnt_t[g] = t2;
    }
  }
}

// The refresh-mode walk, S lanes per group cut as in k_walk_c (stretches
// between the ancestors of the deepest cell gd holding the group and past
// their subtrees), with the refresh-mode geometry: each visit reads the
// 16-byte walk record (skip, leaf flag, leaf count) and the cell's moved
// centre and (effective side / theta)^2 from `ctr`; the lanes also record
// the opening-test slacks of the group (smallest margin of an accepted and
// of an opened cell that does not hold the group) and its cell's shift.
// The cut needs only that ancestors of gd hold the group and are opened,
// which the moved geometry keeps (a cell holding the group's particle range
// is always opened).  The construction walk of refresh mode (sel NULL, slot
// t = group t) and the refresh of a selection (slot t = group sel[t], only
// the first *n_dev slots) are this kernel.  Counts and state go to slot t;
// lane h's token count to cnt_tl[S t + h].  Tokens (FILL) go to
//   lane_off given: the group's lane range [lane_off[S g + h],
//                   lane_off[S g + h + 1]) (the refresh's per-lane room),
//   slab > 0:       slab S t + h of `slab` tokens,
//   else:           after the tokens of lanes 0 .. h - 1 from tok_off[t]
//                   (exact fill after a count pass, counts left as they are).
// Tokens past a lane's room are dropped; its count says so.
template <bool FILL, int S>
__global__ void __launch_bounds__(kWalkThreads)
k_walk_r(int64_t n_walk, int64_t nblk, const uint32_t* __restrict__ sel,
         const uint32_t* __restrict__ n_dev,
         const uint32_t* __restrict__ g_begin,
         const uint32_t* __restrict__ g_count,
         const double4* __restrict__ g_lo, const double4* __restrict__ g_hi,
         const uint32_t* __restrict__ g_cell, const CellRec* __restrict__ rec,
         const uint4* __restrict__ wrec, const double4* __restrict__ ctr,
         const double4* __restrict__ shift, const uint32_t* __restrict__ seg,
         const uint32_t* __restrict__ croot, uint32_t* __restrict__ cnt_e,
         uint32_t* __restrict__ cnt_s, uint32_t* __restrict__ cnt_t,
         uint32_t* __restrict__ cnt_tl, double* __restrict__ o_sa,
         double* __restrict__ o_so, double4* __restrict__ o_tau0,
         const uint64_t* __restrict__ lane_off,
         const uint64_t* __restrict__ tok_off, uint32_t* __restrict__ tok,
         uint32_t slab) {
  static_assert(S == 2 || S == 4 || S == 8, "lanes per group");
  constexpr int H = S / 2;
  __shared__ uint32_t stage[FILL ? kSeg : 1][kWalkThreads];
  const int64_t n_sel =
      (n_dev && (int64_t)*n_dev < n_walk) ? (int64_t)*n_dev : n_walk;
  const int64_t nact = active_blocks(nblk, n_walk, n_dev, kWalkThreads / S);
  const int64_t blk = xcd_block(nact);
  if (blk >= nact) return;
  const int64_t tt = blk * kWalkThreads + threadIdx.x;
  if (tt >= n_sel * S) return;  // the S lanes of a slot leave together
  const int64_t t = tt / S;
  const int h = (int)(tt % S);
  const uint32_t g = sel ? sel[t] : (uint32_t)t;
  const uint32_t gb = g_begin[g];
  const uint32_t ge = gb + g_count[g];
  const double4 lo = g_lo[g], hi = g_hi[g];
  uint32_t gd = g_cell[g];
  for (;;) {
    if ((rec[gd].meta.w >> 8) & 1u) break;
    const uint4 m1 = rec[gd + 1].meta;
    if (m1.x != gb || m1.y != ge) break;
    ++gd;
  }
  const uint32_t sys = seg[gb];
  const uint32_t r0 = croot[sys], r1 = croot[sys + 1];
  uint32_t c, nc;
  if (S == 2) {
    c = h ? gd : r0;
    nc = h ? r1 : gd;
  } else {
    const int D = (int)(rec[gd].meta.w & 255u);
    uint32_t a[H + 1];
    a[0] = r0;
    a[H] = gd;
    uint32_t x = gd;
    int lx = D;
#pragma unroll
    for (int q = H - 1; q >= 1; --q) {
      const int want = (D * q) / H;
      while (lx > want) {
        x = rec[x].aux.x;
        --lx;
      }
      a[q] = x;
    }
    if (h < H) {
      c = a[h];
      nc = a[h + 1];
    } else {
      const int k2 = h - H;
      c = k2 == 0 ? gd : wrec[a[H - k2]].z;
      nc = k2 == H - 1 ? r1 : wrec[a[H - 1 - k2]].z;
    }
  }
  uint64_t out = 0, end = ~0ull;
  if (FILL) {
    if (lane_off) {
      out = lane_off[(uint64_t)g * S + h];
      end = lane_off[(uint64_t)g * S + h + 1];
    } else if (slab) {
      out = ((uint64_t)t * S + (uint64_t)h) * slab;
      end = out + slab;
    } else {
      out = tok_off[t];
      for (int q = 0; q < h; ++q) out += cnt_tl[(uint64_t)t * S + q];
    }
  }
  const bool counts = !FILL || lane_off || slab;
  int sc = 0;
  double sa = __builtin_inf(), so = __builtin_inf();
  uint32_t ne = 0, ns = 0, nl = 0;
  while (c < nc) {
    const uint4 w = wrec[c];
    const double4 cc = ctr[c];
    const uint32_t skip = w.z;
    const bool leaf = (w.y >> 31) != 0u;
    const bool holds = c <= gd && gd < skip;
    double dx = 0.0, dy = 0.0, dz = 0.0, u;
    u = __dsub_rn(lo.x, cc.x);
    if (u > dx) dx = u;
    u = __dsub_rn(cc.x, hi.x);
    if (u > dx) dx = u;
    u = __dsub_rn(lo.y, cc.y);
    if (u > dy) dy = u;
    u = __dsub_rn(cc.y, hi.y);
    if (u > dy) dy = u;
    u = __dsub_rn(lo.z, cc.z);
    if (u > dz) dz = u;
    u = __dsub_rn(cc.z, hi.z);
    if (u > dz) dz = u;
    const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                __dmul_rn(dz, dz));
    const bool open = holds || !(d2 > cc.w);
    if (counts && !holds) {
      const double dd = __dsqrt_rn(d2), rr = __dsqrt_rn(cc.w);
      if (open) {
        const double v = __dsub_rn(rr, dd);
        if (v < so) so = v;
      } else {
        const double v = __dsub_rn(dd, rr);
        if (v < sa) sa = v;
      }
    }
    const bool term = !open || leaf;
    // skip ids always point past the cell; the guard keeps a damaged tree
    // from looping forever
    const uint32_t next = term ? skip : c + 1;
    if (next <= c) break;
    if (term) {
      if (!open) {
        ++ns;
      } else {
        ++nl;
        uint32_t cnt = w.w >> 5;
        if (cnt == kWalkCountSat) cnt = rec[c].meta.y - rec[c].meta.x;
        ne += cnt;
      }
      if (FILL) {
        stage[sc][threadIdx.x] = open ? (c | kLeafTag) : c;
        ++sc;
        if (((out + sc) & (kSeg - 1)) == 0) {
          if (out + sc > end) {
            // past the lane's room: drop
          } else if (sc == kSeg) {
            uint4* d4 = reinterpret_cast<uint4*>(tok + out);
#pragma unroll
            for (int q = 0; q < kSeg / 4; ++q)
              d4[q] = make_uint4(stage[4 * q][threadIdx.x],
                                 stage[4 * q + 1][threadIdx.x],
                                 stage[4 * q + 2][threadIdx.x],
                                 stage[4 * q + 3][threadIdx.x]);
          } else {
            for (int q = 0; q < sc; ++q) tok[out + q] = stage[q][threadIdx.x];
          }
          out += sc;
          sc = 0;
        }
      }
    }
    c = next;
  }
  if (FILL && out + sc <= end)
    for (int q = 0; q < sc; ++q) tok[out + q] = stage[q][threadIdx.x];
  if (!counts) return;  // after the exact fill: uniform over the S lanes
  const uint32_t ta = ns + nl;
  cnt_tl[(uint64_t)t * S + h] = ta;
  uint32_t e2 = ne, s2 = ns, t2 = ta;
#pragma unroll
  for (int o = S / 2; o > 0; o >>= 1) {
    e2 += __shfl_xor(e2, o, 64);
    s2 += __shfl_xor(s2, o, 64);
    t2 += __shfl_xor(t2, o, 64);
    sa = fmin(sa, __shfl_xor(sa, o, 64));
    so = fmin(so, __shfl_xor(so, o, 64));
  }
  if (h == 0) {
    cnt_e[t] = e2;
    cnt_s[t] = s2;
    cnt_t[t] = t2;
    o_sa[t] = sa;
    o_so[t] = so;
    o_tau0[t] = shift[g_cell[g]];
  }
}

// Tile walk: W lanes per group (W = 4 .. 64, a power of two), for more
// parallelism than one thread per group.  The lanes of a tile take W
// consecutive cells of the pre-order array and evaluate the opening test of
// each; a cell is one the stackless walk visits unless an earlier cell of
// the window that ends the walk there (accepted, or an opened leaf) has a
// subtree reaching past it -- an exclusive prefix maximum of those subtree
// ends over the tile.  (Earlier windows cannot hide a cell: the window
// starts at a visited cell, whose ancestors were all opened.)  The next
// window starts at the later of the window's end and the farthest such
// subtree end.  Tokens come out in pre-order, exactly as from the
// one-thread walk.  Small tiles waste little work on cells hidden inside a
// window; large tiles give more lanes when there are few groups.
// slab > 0 (fill pass only): counts and tokens in one pass, the tokens into
// `slab` slots per group, as in the one-thread walk.
template <int W, bool FILL>
__global__ void __launch_bounds__(256)
k_walk_tile(int64_t n_walk, int64_t nblk, const uint32_t* __restrict__ g_begin,
            const uint32_t* __restrict__ g_count,
            const double4* __restrict__ g_lo, const double4* __restrict__ g_hi,
            const CellRec* __restrict__ rec, const uint32_t* __restrict__ seg,
            const uint32_t* __restrict__ croot, uint32_t* __restrict__ cnt_e,
            uint32_t* __restrict__ cnt_s, uint32_t* __restrict__ cnt_t,
            const uint64_t* __restrict__ tok_off, uint32_t* __restrict__ tok,
            uint32_t slab) {
  static_assert(W >= 2 && W <= 64 && (W & (W - 1)) == 0, "tile width");
  const int64_t blk = xcd_block(nblk);
  if (blk >= nblk) return;
  const int64_t t = blk * (256 / W) + (threadIdx.x / W);
  const int lane = threadIdx.x & (W - 1);
  if (t >= n_walk) return;  // uniform over the tile
  const int64_t g = t;
  const uint32_t gb = g_begin[g];
  const uint32_t ge = gb + g_count[g];
  const double4 lo = g_lo[g], hi = g_hi[g];
  // this tile's bits of a wave ballot, and the lanes below this one
  const int base = (int)(threadIdx.x & 63) & ~(W - 1);
  const uint64_t tmask = W == 64 ? ~0ull : ((1ull << W) - 1ull);
  const uint64_t below = lane == 0 ? 0ull : ((1ull << lane) - 1ull);
  uint64_t out = 0, end = ~0ull;
  if (FILL) {
    out = slab ? (uint64_t)t * slab : tok_off[t];
    if (slab) end = out + slab;
  }
  const bool counts = !FILL || slab != 0;
  uint32_t ne = 0, ns = 0, nl = 0;  // per lane
  const uint32_t sys = seg[gb];
  uint32_t c = croot[sys];
  const uint32_t nc = croot[sys + 1];
  while (c < nc) {
    const uint32_t i = c + (uint32_t)lane;
    const bool valid = i < nc;
    uint4 m = make_uint4(0u, 0u, 0u, 0u);
    bool open = false, stop = false;
    if (valid) {
      m = rec[i].meta;
      const double4 cc = rec[i].geo;
      if (m.x <= gb && m.y >= ge) {
        open = true;
      } else {
        double dx = 0.0, dy = 0.0, dz = 0.0, u;
        u = __dsub_rn(lo.x, cc.x);
        if (u > dx) dx = u;
        u = __dsub_rn(cc.x, hi.x);
        if (u > dx) dx = u;
        u = __dsub_rn(lo.y, cc.y);
        if (u > dy) dy = u;
        u = __dsub_rn(cc.y, hi.y);
        if (u > dy) dy = u;
        u = __dsub_rn(lo.z, cc.z);
        if (u > dz) dz = u;
        u = __dsub_rn(cc.z, hi.z);
        if (u > dz) dz = u;
        const double d2 =
            __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                      __dmul_rn(dz, dz));
        open = !(d2 > cc.w);
      }
      stop = !open || ((m.w >> 8) & 1u);
    }
    // exclusive prefix maximum of the subtree ends of stopping cells
    uint32_t incl = stop ? m.z : 0u;
#pragma unroll
    for (int d = 1; d < W; d <<= 1) {
      const uint32_t v = __shfl_up(incl, d, W);
      if (lane >= d && v > incl) incl = v;
    }
    uint32_t excl = __shfl_up(incl, 1, W);
    if (lane == 0) excl = 0u;
    const bool visited = valid && !(excl > i);
    const bool acc = visited && !open;
    const bool lf = visited && open && stop;
    if (counts) {
      ns += acc ? 1u : 0u;
      nl += lf ? 1u : 0u;
      ne += lf ? m.y - m.x : 0u;
    }
    if (FILL) {
      const uint64_t me = (__ballot(acc || lf) >> base) & tmask;
      const uint64_t pos = out + (uint64_t)__popcll(me & below);
      if ((acc || lf) && pos < end) tok[pos] = acc ? i : (i | kLeafTag);
      out += (uint64_t)__popcll(me);
    }
    const uint32_t far = __shfl(incl, W - 1, W);
    const uint32_t next = c + (uint32_t)W;
    c = far > next ? far : next;
  }
  if (counts) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) {
      ne += __shfl_xor(ne, o, W);
      ns += __shfl_xor(ns, o, W);
      nl += __shfl_xor(nl, o, W);
    }
    if (lane == 0) {
      cnt_e[t] = ne;
      cnt_s[t] = ns;
      cnt_t[t] = ns + nl;
    }
  }
}

// One wave per group: the token stream -> SPJ ids and EPJ particle ids.
// Tokens are read in chunks of 64; accepted cells are compacted with a
// ballot, opened leaves are expanded using a wave scan of their sizes, so
// every chunk lands in contiguous stretches of both lists.
// Token offsets and counts are per walked group (index t), except the
// per-lane ranges lane_off, which belong to the group id like the output
// offsets (sel[t], or t when sel is NULL).  With n_dev only the first
// *n_dev slots are expanded, and with ok only the slots t with ok[t].
__global__ void __launch_bounds__(256)
k_expand(int64_t n_walk, int64_t nblk, const uint32_t* __restrict__ sel,
         const uint64_t* __restrict__ tok_off,
         const uint64_t* __restrict__ lane_off, uint32_t slab,
         const uint32_t* __restrict__ cnt_t,
         const uint32_t* __restrict__ cnt_tl, int lanes,
         const uint32_t* __restrict__ tok, const CellRec* __restrict__ rec,
         const uint64_t* __restrict__ epj_off,
         const uint64_t* __restrict__ spj_off, uint32_t* __restrict__ epj,
         uint32_t* __restrict__ spj, const uint32_t* __restrict__ n_dev,
         const uint8_t* __restrict__ ok) {
  const int64_t nact = active_blocks(nblk, n_walk, n_dev, 4);
  const int64_t blk = xcd_block(nact);
  if (blk >= nact) return;
  const int64_t t = blk * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= n_walk || (n_dev && t >= (int64_t)*n_dev) || (ok && !ok[t]))
    return;  // uniform over the wave
  const int64_t g = sel ? (int64_t)sel[t] : t;
  // the token stream: one range, or (a walk with `lanes` lanes per group
  // whose tokens sit in per-lane slabs or per-lane ranges, cnt_tl given)
  // the lanes' ranges one after the other
  const int nr = ((slab || lane_off) && cnt_tl) ? lanes : 1;
  uint64_t oe = epj_off[g], os = spj_off[g];
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  // kExpandBatch chunks of 64 tokens per round: their token loads, then
  // their leaves' record loads, are issued together, so a round waits for
  // two memory latencies instead of two per chunk
  for (int ri = 0; ri < nr; ++ri) {
    uint64_t t0, t1;
    if (lane_off) {
      t0 = lane_off[(uint64_t)g * (uint64_t)lanes + (uint64_t)ri];
      t1 = t0 + cnt_tl[(uint64_t)t * (uint64_t)lanes + (uint64_t)ri];
    } else if (!slab) {
      t0 = tok_off[t];
      t1 = tok_off[t + 1];
    } else if (!cnt_tl) {
      t0 = (uint64_t)t * slab;
      t1 = t0 + cnt_t[t];
    } else {
      t0 = ((uint64_t)t * (uint64_t)lanes + (uint64_t)ri) * slab;
      t1 = t0 + cnt_tl[(uint64_t)t * (uint64_t)lanes + (uint64_t)ri];
    }
    for (uint64_t cb = t0; cb < t1; cb += 64 * kExpandBatch) {
      uint32_t tk[kExpandBatch], bb[kExpandBatch], nn[kExpandBatch];
#pragma unroll
      for (int u = 0; u < kExpandBatch; ++u) {
        const uint64_t q = cb + 64 * u + lane;
        tk[u] = q < t1 ? tok[q] : 0u;
      }
#pragma unroll
      for (int u = 0; u < kExpandBatch; ++u) {
        const uint64_t q = cb + 64 * u + lane;
        bb[u] = 0;
        nn[u] = 0;
        if (q < t1 && (tk[u] & kLeafTag)) {
          const uint4 m = rec[tk[u] & ~kLeafTag].meta;
          bb[u] = m.x;
          nn[u] = m.y - m.x;
        }
      }
#pragma unroll
      for (int u = 0; u < kExpandBatch; ++u) {
        const bool ok = cb + 64 * u + lane < t1;
        const bool is_spj = ok && !(tk[u] & kLeafTag);
        const uint64_t sm = __ballot(is_spj);
        if (is_spj) spj[os + __popcll(sm & lt)] = tk[u];
        os += __popcll(sm);
        const uint32_t n = nn[u], b = bb[u];
        uint32_t inc = n;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t v = __shfl_up(inc, d, 64);
          if (lane >= d) inc += v;
        }
        const uint32_t total = __shfl(inc, 63, 64);
        // the chunk's particle ids, written by the whole wave in contiguous
        // runs of 64: entry k belongs to the first lane whose inclusive
        // size sum exceeds k (a binary search over the lanes' sums)
        for (uint32_t k0 = 0; k0 < total; k0 += 64) {
          const uint32_t k = k0 + (uint32_t)lane;
          int L = 0;
#pragma unroll
          for (int step = 32; step > 0; step >>= 1)
            if (__shfl(inc, L + step - 1, 64) <= k) L += step;
          const uint32_t first = __shfl(b, L, 64);
          const uint32_t before = __shfl(inc - n, L, 64);
          if (k < total) epj[oe + k] = first + (k - before);
        }
        oe += total;
      }
    }
  }
}

// Interactions of the lists: sum over groups of n_i * (n_epj + n_spj) into
// out[0], of n_i * n_spj (superparticle interactions) into out[2], and the
// list entries into out[4] (particles) and out[5] (superparticles).
__global__ void __launch_bounds__(256)
k_interactions(int64_t n_groups, const uint32_t* __restrict__ g_count,
               const uint32_t* __restrict__ cnt_e,
               const uint32_t* __restrict__ cnt_s,
               unsigned long long* __restrict__ out) {
  __shared__ unsigned long long s[4][4];
  unsigned long long v[4] = {0, 0, 0, 0};
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
       g < n_groups; g += (int64_t)gridDim.x * blockDim.x) {
    v[0] += (unsigned long long)g_count[g] *
            ((unsigned long long)cnt_e[g] + cnt_s[g]);
    v[1] += (unsigned long long)g_count[g] * cnt_s[g];
    v[2] += cnt_e[g];
    v[3] += cnt_s[g];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    if ((threadIdx.x & 63) == 0) s[q][threadIdx.x >> 6] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int dst[4] = {kRedInter, kRedInterSpj, kRedEpj, kRedSpj};
#pragma unroll
    for (int q = 0; q < 4; ++q)
      atomicAdd(out + dst[q], (s[q][0] + s[q][1]) + (s[q][2] + s[q][3]));
  }
}

// List slots of refresh mode: three times the list plus the mean list
// length of the construction (red[kRedEpj] / groups, plus 32), so that
// short lists can grow to typical ones.
__global__ void __launch_bounds__(256)
k_slot_caps(int64_t n_groups, const uint32_t* __restrict__ cnt_e,
            const uint32_t* __restrict__ cnt_s,
            const unsigned long long* __restrict__ red,
            uint32_t* __restrict__ cap_e, uint32_t* __restrict__ cap_s) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const uint64_t me = red[kRedEpj] / (uint64_t)n_groups + 32u;
  const uint64_t ms = red[kRedSpj] / (uint64_t)n_groups + 32u;
  const uint64_t ce = 3u * (uint64_t)cnt_e[g] + me;
  const uint64_t cs = 3u * (uint64_t)cnt_s[g] + ms;
  cap_e[g] = ce < 0xFFFFFFFFull ? (uint32_t)ce : 0xFFFFFFFFu;
  cap_s[g] = cs < 0xFFFFFFFFull ? (uint32_t)cs : 0xFFFFFFFFu;
}

// Room of each refresh-walk lane: twice its tokens at construction plus
// kLaneSpare, rounded up to whole 64-byte segments.
__global__ void __launch_bounds__(256)
k_lane_room(int64_t n, const uint32_t* __restrict__ cnt_tl,
            uint32_t* __restrict__ cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t r = (2ull * cnt_tl[i] + kLaneSpare + 15ull) & ~15ull;
  cap[i] = r < 0xFFFFFFF0ull ? (uint32_t)r : 0xFFFFFFF0u;
}

// Per-force-call counters of refresh mode (see kRed*).
__global__ void k_accum(unsigned long long* __restrict__ red,
                        int refresh_step) {
  if (threadIdx.x != 0) return;
  red[kRedTotInter] += red[kRedInter];
  red[kRedTotInterSpj] += red[kRedInterSpj];
  if (refresh_step) {
    red[kRedTotRefreshed] += red[kRedRefreshed];
    red[kRedTotOverflow] += red[kRedOverflow];
  } else {
    red[kRedRefreshed] = 0ull;
    red[kRedOverflow] = 0ull;
  }
}

// Largest per-group token count into *out (zeroed before).
__global__ void __launch_bounds__(256)
k_max_u32(int64_t n, const uint32_t* __restrict__ v,
          unsigned long long* __restrict__ out) {
  unsigned long long m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = v[i] > m ? v[i] : m;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long u = __shfl_xor(m, o, 64);
    m = u > m ? u : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// Short-range walk (section 2: the same group walk with another opening
// rule; reuse as in section 4.2).  A cell that holds the group is opened;
// any other cell when its cube overlaps the group's tight box grown by h on
// every side: on each axis the gap between the box and the cell's centre
// (zero inside) is at most half the cell's side plus h.  Cells that fail
// are skipped with their subtree; an opened leaf becomes a token, expanded
// into its particles as for the gravity lists.  FP64, explicit rounding.
// Two lanes per group, split at gd as in the gravity walk; the count pass
// records the first half's tokens (cnt_ta) so the fill's second half writes
// after them.
template <bool FILL>
__global__ void __launch_bounds__(kWalkThreads)
k_walk_nbr(int64_t n_walk, int64_t nblk, const uint32_t* __restrict__ g_begin,
           const uint32_t* __restrict__ g_count,
           const double4* __restrict__ g_lo, const double4* __restrict__ g_hi,
           const uint32_t* __restrict__ g_cell,
           const CellRec* __restrict__ rec, const uint4* __restrict__ wrec,
           const uint32_t* __restrict__ seg,
           const uint32_t* __restrict__ croot, const Root* __restrict__ root,
           double h, uint32_t* __restrict__ cnt_e,
           uint32_t* __restrict__ cnt_t, uint32_t* __restrict__ cnt_ta,
           const uint64_t* __restrict__ tok_off,
           uint32_t* __restrict__ tok) {
  __shared__ uint32_t stage[FILL ? kSeg : 1][kWalkThreads];
  const int64_t blk = xcd_block(nblk);
  if (blk >= nblk) return;
  // two lanes per group, split at gd as in the gravity walk (n_walk = 2 x
  // groups: the lanes of a group leave together)
  const int64_t tt = blk * kWalkThreads + threadIdx.x;
  if (tt >= n_walk) return;
  const int64_t g = tt >> 1;
  const int half = (int)(tt & 1);
  const uint32_t gb = g_begin[g];
  const uint32_t ge = gb + g_count[g];
  const double4 lo = g_lo[g], hi = g_hi[g];
  // deepest cell whose range is the group's (as in the gravity walk)
  uint32_t gd = g_cell[g];
  for (;;) {
    if ((rec[gd].meta.w >> 8) & 1u) break;
    const uint4 m1 = rec[gd + 1].meta;
    if (m1.x != gb || m1.y != ge) break;
    ++gd;
  }
  const uint32_t sys = seg[gb];
  const Root* rt = root + sys;
  const double rx = rt->lo[0], ry = rt->lo[1], rz = rt->lo[2];
  const int k = rt->k;
  uint32_t c = half ? gd : croot[sys];
  const uint32_t nc = half ? croot[sys + 1] : gd;
  uint64_t out = FILL ? tok_off[g] + (half ? cnt_ta[g] : 0u) : 0;
  int sc = 0;
  uint32_t ne = 0, nl = 0;
  // the gravity walk's visit: one record load, no divergent branch, full
  // token segments stored one visit late
  asm volatile("" ::"v"(c), "v"(nc), "v"(gd), "v"(k), "v"(rx), "v"(ry),
               "v"(rz));
  asm volatile("" ::"v"(lo.x), "v"(lo.y), "v"(lo.z), "v"(hi.x), "v"(hi.y),
               "v"(hi.z), "v"(gb));
  uint4 seg0, seg1, seg2, seg3;
  uint32_t* pend = nullptr;
  while (c < nc) {
    const uint4 w = wrec[c];
    asm volatile("" ::"v"(w.x), "v"(w.y), "v"(w.z), "v"(w.w));
    if (FILL && pend) {
      uint4* d4 = reinterpret_cast<uint4*>(pend);
      d4[0] = seg0;
      d4[1] = seg1;
      d4[2] = seg2;
      d4[3] = seg3;
      pend = nullptr;
    }
    const uint32_t skip = w.z;
    const bool leaf = (w.y >> 31) != 0u;
    const int l = (int)(w.w & 31u);
    const uint64_t q = (uint64_t)w.x | ((uint64_t)(w.y & 0x7FFFFFFFu) << 32);
    const uint32_t qx = (uint32_t)q & 0x1FFFFFu;
    const uint32_t qy = (uint32_t)(q >> 21) & 0x1FFFFFu;
    const uint32_t qz = (uint32_t)(q >> 42);
    const double half = ldexp(1.0, k - l - 1);
    const double cx = __dadd_rn(rx, __dmul_rn((double)(2u * qx + 1u), half));
    const double cy = __dadd_rn(ry, __dmul_rn((double)(2u * qy + 1u), half));
    const double cz = __dadd_rn(rz, __dmul_rn((double)(2u * qz + 1u), half));
    // the cube grown by h overlaps the group's box on every axis
    const double r = __dadd_rn(half, h);
    const double vx = fmax(fmax(__dsub_rn(lo.x, cx), __dsub_rn(cx, hi.x)), 0.0);
    const double vy = fmax(fmax(__dsub_rn(lo.y, cy), __dsub_rn(cy, hi.y)), 0.0);
    const double vz = fmax(fmax(__dsub_rn(lo.z, cz), __dsub_rn(cz, hi.z)), 0.0);
    const bool open = (c <= gd && gd < skip) ||
                      (!(vx > r) && !(vy > r) && !(vz > r));
    const uint32_t next = (!open || leaf) ? skip : c + 1;
    if (next <= c) break;
    const bool opened_leaf = open && leaf;
    uint32_t cnt = w.w >> 5;
    if (cnt == kWalkCountSat) cnt = rec[c].meta.y - rec[c].meta.x;
    nl += opened_leaf ? 1u : 0u;
    ne += opened_leaf ? cnt : 0u;
    if (FILL) {
      stage[sc][threadIdx.x] = c | kLeafTag;
      sc += opened_leaf ? 1 : 0;
      if (opened_leaf && ((out + sc) & (kSeg - 1)) == 0) {
        if (sc == kSeg) {
          seg0 = make_uint4(stage[0][threadIdx.x], stage[1][threadIdx.x],
                            stage[2][threadIdx.x], stage[3][threadIdx.x]);
          seg1 = make_uint4(stage[4][threadIdx.x], stage[5][threadIdx.x],
                            stage[6][threadIdx.x], stage[7][threadIdx.x]);
          seg2 = make_uint4(stage[8][threadIdx.x], stage[9][threadIdx.x],
                            stage[10][threadIdx.x], stage[11][threadIdx.x]);
          seg3 = make_uint4(stage[12][threadIdx.x], stage[13][threadIdx.x],
                            stage[14][threadIdx.x], stage[15][threadIdx.x]);
          pend = tok + out;
        } else {
          for (int t = 0; t < sc; ++t) tok[out + t] = stage[t][threadIdx.x];
        }
        out += sc;
        sc = 0;
      }
    }
    c = next;
  }
  if (FILL) {
    if (pend) {
      uint4* d4 = reinterpret_cast<uint4*>(pend);
      d4[0] = seg0;
      d4[1] = seg1;
      d4[2] = seg2;
      d4[3] = seg3;
    }
    for (int t = 0; t < sc; ++t) tok[out + t] = stage[t][threadIdx.x];
  } else {
    const uint32_t e2 = ne + __shfl_xor(ne, 1, 64);
    const uint32_t t2 = nl + __shfl_xor(nl, 1, 64);
    if (half == 0) {
      cnt_e[g] = e2;
      cnt_t[g] = t2;
      cnt_ta[g] = nl;
    }
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// Caller-supplied CSR offsets (n_groups + 1 values): they must start at 0,
// never decrease, end at the declared total, and give no group 2^32 or more
// entries.  Sets `bit` in *flag otherwise; writes each group's length to
// cnt (0 where the offsets are bad).  Reads only the offsets.
__global__ void __launch_bounds__(256)
k_check_offsets(int64_t ng, const uint64_t* __restrict__ off, uint64_t total,
                uint32_t* __restrict__ cnt, unsigned bit,
                unsigned* __restrict__ flag) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g > ng) return;
  bool bad = false;
  if (g == 0 && off[0] != 0ull) bad = true;
  if (g == ng) {
    if (off[ng] != total) bad = true;
  } else {
    const uint64_t a = off[g], b = off[g + 1];
    const bool ok = b >= a && b - a < 0xFFFFFFFFull;
    cnt[g] = ok ? (uint32_t)(b - a) : 0u;
    if (!ok) bad = true;
  }
  if (bad) atomicOr(flag, bit);
}

// Ids of caller-supplied lists against their bound (particle slots < n,
// cell ids < n_cell).  Sets `bit` in *flag if any is out of range; reads
// only the n ids.
__global__ void __launch_bounds__(256)
k_check_ids(int64_t n, const uint32_t* __restrict__ id, uint32_t limit,
            unsigned bit, unsigned* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= id[i] >= limit;
  if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, bit);
}

}  // namespace

// Check caller-supplied lists already copied into epj_off/epj/spj_off/spj
// (totals n_epj, n_spj): flag bits 1 / 2 = bad EPJ / SPJ offsets, 4 / 8 =
// EPJ / SPJ id out of range; per-group lengths into cnt_e, cnt_s.
int launch_check_lists(nb_ctx* c, unsigned* flag) {
  const unsigned nb = grid_for(c->n_groups + 1, 256);
  hipLaunchKernelGGL(k_check_offsets, dim3(nb), dim3(256), 0, c->stream,
                     c->n_groups, (const uint64_t*)c->epj_off.p,
                     (uint64_t)c->n_epj, c->cnt_e.p, 1u, flag);
  hipLaunchKernelGGL(k_check_offsets, dim3(nb), dim3(256), 0, c->stream,
                     c->n_groups, (const uint64_t*)c->spj_off.p,
                     (uint64_t)c->n_spj, c->cnt_s.p, 2u, flag);
  unsigned ne = grid_for(c->n_epj, 256), ns = grid_for(c->n_spj, 256);
  if (ne > 2048) ne = 2048;
  if (ns > 2048) ns = 2048;
  hipLaunchKernelGGL(k_check_ids, dim3(ne), dim3(256), 0, c->stream,
                     c->n_epj, (const uint32_t*)c->epj.p, (uint32_t)c->n, 4u,
                     flag);
  hipLaunchKernelGGL(k_check_ids, dim3(ns), dim3(256), 0, c->stream,
                     c->n_spj, (const uint32_t*)c->spj.p,
                     (uint32_t)c->n_cell, 8u, flag);
  return hip_check(c, hipGetLastError(), "list check launch");
}

// Whether a walk over n_walk groups runs kSplitLanes lanes per group
// (k_walk_c, and k_walk_r in refresh mode), whose slab mode takes that many
// slabs per group.
bool split_walk(const nb_ctx* c, int64_t n_walk) {
  return c->learn || walk_tile(n_walk) == 1;
}

// Lanes per tile of a walk over n_walk groups (1: split walk; see
// kThreadWalkFrom).
int walk_tile(int64_t n_walk) {
  if (n_walk >= kThreadWalkFrom) return 1;
  int w = kTileWalk;
  while (w < 64 && (int64_t)w * n_walk < kTileLanes) w <<= 1;
  return w;
}

template <int W>
static void tile_launch(nb_ctx* c, bool fill, int64_t launch, int64_t n_walk,
                        int64_t nblk, const double4* lo, const double4* hi,
                        uint32_t slab) {
  auto k = fill ? k_walk_tile<W, true> : k_walk_tile<W, false>;
  hipLaunchKernelGGL(k, dim3((unsigned)launch), dim3(256), 0, c->stream,
                     n_walk, nblk, (const uint32_t*)c->g_begin.p,
                     (const uint32_t*)c->g_count.p, lo, hi,
                     (const CellRec*)c->c_rec.p, (const uint32_t*)c->seg.p,
                     (const uint32_t*)c->croot.p, c->cnt_e.p, c->cnt_s.p,
                     c->cnt_t.p, (const uint64_t*)c->tok_off.p, c->tok.p,
                     slab);
}

static void launch_tile(nb_ctx* c, int w, bool fill, int64_t launch,
                        int64_t n_walk, int64_t nblk, const double4* lo,
                        const double4* hi, uint32_t slab) {
  switch (w) {
    case 4: tile_launch<4>(c, fill, launch, n_walk, nblk, lo, hi, slab); break;
    case 8: tile_launch<8>(c, fill, launch, n_walk, nblk, lo, hi, slab); break;
    case 16: tile_launch<16>(c, fill, launch, n_walk, nblk, lo, hi, slab); break;
    case 32: tile_launch<32>(c, fill, launch, n_walk, nblk, lo, hi, slab); break;
    default: tile_launch<64>(c, fill, launch, n_walk, nblk, lo, hi, slab); break;
  }
}

// k_walk_r over n_walk slots (selected groups when sel is given, their
// number *o.n_dev on the device), outputs as o says.
static void launch_walk_r(nb_ctx* c, bool fill, int64_t n_walk,
                          const uint32_t* sel, const double4* lo,
                          const double4* hi, const WalkOut& o,
                          const uint64_t* lane_off, uint32_t slab) {
  const int64_t nblk = grid_for(kSplitLanes * n_walk, kWalkThreads);
  const int64_t launch = (nblk + 7) / 8 * 8;
  auto k = fill ? k_walk_r<true, kSplitLanes> : k_walk_r<false, kSplitLanes>;
  hipLaunchKernelGGL(k, dim3((unsigned)launch), dim3(kWalkThreads), 0,
                     c->stream, n_walk, nblk, sel, o.n_dev,
                     (const uint32_t*)c->g_begin.p,
                     (const uint32_t*)c->g_count.p, lo, hi,
                     (const uint32_t*)c->g_cell.p, (const CellRec*)c->c_rec.p,
                     (const uint4*)c->c_wrec.p, (const double4*)c->c_ctr.p,
                     (const double4*)c->c_shift.p, (const uint32_t*)c->seg.p,
                     (const uint32_t*)c->croot.p, o.cnt_e, o.cnt_s, o.cnt_t,
                     c->cnt_tl.p, o.sa, o.so, o.tau0, lane_off,
                     (const uint64_t*)c->tok_off.p, c->tok.p, slab);
}

int launch_walk_refresh(nb_ctx* c, int64_t n_max, const uint32_t* sel,
                        const double4* lo, const double4* hi,
                        const WalkOut& o) {
  if (c->n_cell >= (int64_t)kLeafTag)
    return set_err(c, NB_ERR_INPUT, "too many cells for 31-bit list tokens");
  if (n_max <= 0) return NB_OK;
  launch_walk_r(c, true, n_max, sel, lo, hi, o,
                (const uint64_t*)c->lane_off.p, 0u);
  return hip_check(c, hipGetLastError(), "refresh walk launch");
}

int launch_expand_sel(nb_ctx* c, int64_t n_max, const uint32_t* sel,
                      const uint32_t* n_dev, const uint8_t* ok) {
  if (n_max <= 0) return NB_OK;
  const int64_t eblk = grid_for(n_max, 4);
  const int64_t elaunch = (eblk + 7) / 8 * 8;
  hipLaunchKernelGGL(k_expand, dim3((unsigned)elaunch), dim3(256), 0,
                     c->stream, n_max, eblk, sel, (const uint64_t*)nullptr,
                     (const uint64_t*)c->lane_off.p, 0u,
                     (const uint32_t*)nullptr, (const uint32_t*)c->cnt_tl.p,
                     kSplitLanes, (const uint32_t*)c->tok.p,
                     (const CellRec*)c->c_rec.p,
                     (const uint64_t*)c->epj_off.p,
                     (const uint64_t*)c->spj_off.p, c->epj.p, c->spj.p, n_dev,
                     ok);
  return hip_check(c, hipGetLastError(), "refresh expand launch");
}

int launch_walk(nb_ctx* c, bool fill, uint32_t slab) {
  const size_t ng = (size_t)c->n_groups;
  int rc = reserve(c, c->cnt_e, ng);
  if (!rc) rc = reserve(c, c->cnt_s, ng);
  if (!rc) rc = reserve(c, c->cnt_t, ng);
  if (!rc) rc = reserve(c, c->epj_off, ng + 1);
  if (!rc) rc = reserve(c, c->spj_off, ng + 1);
  if (!rc) rc = reserve(c, c->tok_off, ng + 1);
  if (rc) return rc;
  return launch_walk_sel(c, fill, c->n_groups, c->g_lo.p, c->g_hi.p,
                         c->epj_off.p, c->spj_off.p, c->epj.p, c->spj.p,
                         slab);
}

// Expand of a slab-mode fill pass (tokens at group * slab, counts known).
int launch_expand_slab(nb_ctx* c, uint32_t slab) {
  const int64_t eblk = grid_for(c->n_groups, 4);
  const int64_t elaunch = (eblk + 7) / 8 * 8;
  hipLaunchKernelGGL(k_expand, dim3((unsigned)elaunch), dim3(256), 0,
                     c->stream, c->n_groups, eblk, (const uint32_t*)nullptr,
                     (const uint64_t*)c->tok_off.p, (const uint64_t*)nullptr,
                     slab, (const uint32_t*)c->cnt_t.p,
                     (const uint32_t*)(c->walk_split ? c->cnt_tl.p : nullptr),
                     kSplitLanes, (const uint32_t*)c->tok.p,
                     (const CellRec*)c->c_rec.p,
                     (const uint64_t*)c->epj_off.p,
                     (const uint64_t*)c->spj_off.p, c->epj.p, c->spj.p,
                     (const uint32_t*)nullptr, (const uint8_t*)nullptr);
  return hip_check(c, hipGetLastError(), "expand launch");
}

int launch_walk_sel(nb_ctx* c, bool fill, int64_t n_walk, const double4* lo,
                    const double4* hi, const uint64_t* epj_off,
                    const uint64_t* spj_off, uint32_t* epj, uint32_t* spj,
                    uint32_t slab) {
  if (c->n_cell >= (int64_t)kLeafTag)
    return set_err(c, NB_ERR_INPUT, "too many cells for 31-bit list tokens");
  if (n_walk <= 0) return NB_OK;
  int rc = NB_OK;
  c->walk_split = split_walk(c, n_walk);
  if (c->walk_split &&
      (rc = reserve(c, c->cnt_tl, (size_t)kSplitLanes * n_walk)))
    return rc;
  if (c->learn) {
    // refresh mode: moved-centre geometry, slacks and shifts per group
    const WalkOut o{c->cnt_e.p, c->cnt_s.p, c->cnt_t.p, c->g_sa.p,
                    c->g_so.p, c->g_tau0.p, nullptr};
    launch_walk_r(c, fill, n_walk, nullptr, lo, hi, o, nullptr, slab);
  } else if (!c->walk_split) {
    const int w = walk_tile(n_walk);
    const int64_t nblk = grid_for(n_walk, 256 / w);
    const int64_t launch = (nblk + 7) / 8 * 8;
    launch_tile(c, w, fill, launch, n_walk, nblk, lo, hi, slab);
  } else {
    const int64_t nblk = grid_for(kSplitLanes * n_walk, kWalkThreads);
    const int64_t launch = (nblk + 7) / 8 * 8;
    auto kw = fill ? k_walk_c<true, kSplitLanes>
                   : k_walk_c<false, kSplitLanes>;
    hipLaunchKernelGGL(kw, dim3((unsigned)launch), dim3(kWalkThreads), 0,
                       c->stream, kSplitLanes * n_walk, nblk,
                       (const uint32_t*)c->g_begin.p,
                       (const uint32_t*)c->g_count.p, lo, hi,
                       (const uint32_t*)c->g_cell.p,
                       (const CellRec*)c->c_rec.p, (const uint4*)c->c_wrec.p,
                       (const Root*)c->root.p, (const uint32_t*)c->seg.p,
                       (const uint32_t*)c->croot.p, c->cnt_e.p, c->cnt_s.p,
                       c->cnt_t.p, c->cnt_tl.p, (const uint64_t*)c->tok_off.p,
                       c->tok.p, slab);
  }
  int rc2 = hip_check(c, hipGetLastError(), "walk launch");
  if (rc2 || !fill || slab) return rc2;
  const int64_t eblk = grid_for(n_walk, 4);
  const int64_t elaunch = (eblk + 7) / 8 * 8;
  hipLaunchKernelGGL(k_expand, dim3((unsigned)elaunch), dim3(256), 0,
                     c->stream, n_walk, eblk, (const uint32_t*)nullptr,
                     (const uint64_t*)c->tok_off.p, (const uint64_t*)nullptr,
                     0u, (const uint32_t*)c->cnt_t.p, (const uint32_t*)nullptr,
                     1, (const uint32_t*)c->tok.p, (const CellRec*)c->c_rec.p,
                     epj_off, spj_off, epj, spj, (const uint32_t*)nullptr,
                     (const uint8_t*)nullptr);
  return hip_check(c, hipGetLastError(), "expand launch");
}

// After the count pass: CSR offsets and the interaction count (red[0]).  In
// refresh mode the offsets are those of list slots with room to grow.
int launch_list_stats(nb_ctx* c) {
  int rc = launch_interactions(c, c->cnt_e.p, c->cnt_s.p);
  if (rc) return rc;
  if (c->learn) {
    hipLaunchKernelGGL(k_slot_caps, dim3(grid_for(c->n_groups, 256)),
                       dim3(256), 0, c->stream, c->n_groups,
                       (const uint32_t*)c->cnt_e.p,
                       (const uint32_t*)c->cnt_s.p,
                       (const unsigned long long*)c->red.p, c->ne2.p,
                       c->ns2.p);
    rc = hip_check(c, hipGetLastError(), "slot launch");
    if (!rc) rc = scan_u32_to_u64(c, c->ne2.p, c->epj_off.p, c->n_groups);
    if (!rc) rc = scan_u32_to_u64(c, c->ns2.p, c->spj_off.p, c->n_groups);
  } else {
    rc = scan_u32_to_u64(c, c->cnt_e.p, c->epj_off.p, c->n_groups);
    if (!rc) rc = scan_u32_to_u64(c, c->cnt_s.p, c->spj_off.p, c->n_groups);
  }
  if (!rc) rc = scan_u32_to_u64(c, c->cnt_t.p, c->tok_off.p, c->n_groups);
  if (!rc && c->learn) rc = launch_lane_room(c);
  if (rc) return rc;
  unsigned nb = grid_for(c->n_groups, 256);
  if (nb > 1024) nb = 1024;
  // largest token count of one slab: per lane when the walk ran split
  const bool lanes = c->walk_split;
  hipLaunchKernelGGL(k_max_u32, dim3(nb), dim3(256), 0, c->stream,
                     lanes ? kSplitLanes * c->n_groups : c->n_groups,
                     (const uint32_t*)(lanes ? c->cnt_tl.p : c->cnt_t.p),
                     (unsigned long long*)c->red.p + 1);
  return hip_check(c, hipGetLastError(), "list max launch");
}

int launch_lane_room(nb_ctx* c) {
  const int64_t n = (int64_t)kSplitLanes * c->n_groups;
  int rc = reserve(c, c->lane_cap, (size_t)n);
  if (!rc) rc = reserve(c, c->lane_off, (size_t)n + 1);
  if (rc) return rc;
  hipLaunchKernelGGL(k_lane_room, dim3(grid_for(n, 256)), dim3(256), 0,
                     c->stream, n, (const uint32_t*)c->cnt_tl.p,
                     c->lane_cap.p);
  rc = hip_check(c, hipGetLastError(), "lane room launch");
  return rc ? rc : scan_u32_to_u64(c, c->lane_cap.p, c->lane_off.p, n);
}

int launch_accum(nb_ctx* c, bool refresh_step) {
  hipLaunchKernelGGL(k_accum, dim3(1), dim3(64), 0, c->stream,
                     (unsigned long long*)c->red.p, refresh_step ? 1 : 0);
  return hip_check(c, hipGetLastError(), "counter launch");
}

// Interaction counts of per-group list lengths ne, ns into red[0] (all)
// and red[2] (superparticles), the lengths' sums into red[4] and red[5].
int launch_interactions(nb_ctx* c, const uint32_t* ne, const uint32_t* ns) {
  int rc = reserve(c, c->red, kRedCount);
  if (rc) return rc;
  // the persistent counters start at zero once per allocation
  const bool fresh = c->red_zeroed != c->red.p;
  c->red_zeroed = c->red.p;
  // counters 0-5 describe the current lists; 6-11 persist (all start at 0)
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, c->stream,
                     (unsigned long long*)c->red.p, fresh ? kRedCount : 6);
  unsigned nb = grid_for(c->n_groups, 256);
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_interactions, dim3(nb), dim3(256), 0, c->stream,
                     c->n_groups, (const uint32_t*)c->g_count.p, ne, ns,
                     (unsigned long long*)c->red.p);
  return hip_check(c, hipGetLastError(), "list stats launch");
}


// Short-range walk, count pass: per-group entries and tokens, their CSR
// offsets (nb_off, nb_toff; totals at [n_groups]).
int launch_nbr_count(nb_ctx* c, double h) {
  if (c->n_cell >= (int64_t)kLeafTag)
    return set_err(c, NB_ERR_INPUT, "too many cells for 31-bit list tokens");
  const size_t ng = (size_t)c->n_groups;
  int rc = reserve(c, c->nb_cnt, ng);
  if (!rc) rc = reserve(c, c->nb_tcnt, ng);
  if (!rc) rc = reserve(c, c->nb_tcnt_a, ng);
  if (!rc) rc = reserve(c, c->nb_off, ng + 1);
  if (!rc) rc = reserve(c, c->nb_toff, ng + 1);
  if (rc) return rc;
  // two lanes per group
  const int64_t nblk = grid_for(2 * c->n_groups, kWalkThreads);
  if (nblk > 0)
    hipLaunchKernelGGL(k_walk_nbr<false>, dim3((unsigned)((nblk + 7) / 8 * 8)),
                       dim3(kWalkThreads), 0, c->stream, 2 * c->n_groups,
                       nblk,
                       (const uint32_t*)c->g_begin.p,
                       (const uint32_t*)c->g_count.p,
                       (const double4*)c->g_lo.p, (const double4*)c->g_hi.p,
                       (const uint32_t*)c->g_cell.p,
                       (const CellRec*)c->c_rec.p, (const uint4*)c->c_wrec.p,
                       (const uint32_t*)c->seg.p,
                       (const uint32_t*)c->croot.p, (const Root*)c->root.p, h,
                       c->nb_cnt.p, c->nb_tcnt.p, c->nb_tcnt_a.p,
                       (const uint64_t*)nullptr, (uint32_t*)nullptr);
  if ((rc = hip_check(c, hipGetLastError(), "neighbour walk launch")))
    return rc;
  rc = scan_u32_to_u64(c, c->nb_cnt.p, c->nb_off.p, c->n_groups);
  if (!rc) rc = scan_u32_to_u64(c, c->nb_tcnt.p, c->nb_toff.p, c->n_groups);
  return rc;
}

// Fill pass into c->tok (n tokens reserved) and expand into c->nb_ids.
int launch_nbr_fill(nb_ctx* c, double h) {
  const int64_t nblk = grid_for(2 * c->n_groups, kWalkThreads);
  if (nblk <= 0) return NB_OK;
  hipLaunchKernelGGL(k_walk_nbr<true>, dim3((unsigned)((nblk + 7) / 8 * 8)),
                     dim3(kWalkThreads), 0, c->stream, 2 * c->n_groups, nblk,
                     (const uint32_t*)c->g_begin.p,
                     (const uint32_t*)c->g_count.p,
                     (const double4*)c->g_lo.p, (const double4*)c->g_hi.p,
                     (const uint32_t*)c->g_cell.p,
                     (const CellRec*)c->c_rec.p, (const uint4*)c->c_wrec.p,
                     (const uint32_t*)c->seg.p,
                     (const uint32_t*)c->croot.p, (const Root*)c->root.p, h,
                     (uint32_t*)nullptr, (uint32_t*)nullptr,
                     c->nb_tcnt_a.p, (const uint64_t*)c->nb_toff.p, c->tok.p);
  int rc = hip_check(c, hipGetLastError(), "neighbour fill launch");
  if (rc) return rc;
  // only leaf tokens: the superparticle side of the expand is never written
  const int64_t eblk = grid_for(c->n_groups, 4);
  hipLaunchKernelGGL(k_expand, dim3((unsigned)((eblk + 7) / 8 * 8)),
                     dim3(256), 0, c->stream, c->n_groups, eblk,
                     (const uint32_t*)nullptr, (const uint64_t*)c->nb_toff.p,
                     (const uint64_t*)nullptr, 0u,
                     (const uint32_t*)c->nb_tcnt.p, (const uint32_t*)nullptr,
                     1, (const uint32_t*)c->tok.p, (const CellRec*)c->c_rec.p,
                     (const uint64_t*)c->nb_off.p,
                     (const uint64_t*)c->nb_off.p, c->nb_ids.p,
                     (uint32_t*)nullptr, (const uint32_t*)nullptr,
                     (const uint8_t*)nullptr);
  return hip_check(c, hipGetLastError(), "neighbour expand launch");
}

}  // namespace nb
