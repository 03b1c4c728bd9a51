// nb_walk.hip -- group-wise tree walk emitting index interaction lists
// (section 4.3 list construction; indirect addressing of section 4.1: the
// lists hold 32-bit indices, particles by internal slot, superparticles by
// cell id).
//
// One thread walks one group: a stackless DFS over the pre-order cell array,
// jumping over a subtree with its skip id.  The opening test compares the
// squared distance from the group's tight box to the cell's geometric centre
// with (side / theta)^2 in FP64, evaluated term by term (no fused
// multiply-add: this file is built with -ffp-contract=off and uses explicit
// rounding intrinsics), so that lists are bit-identical to an FP64 reference.
// A cell whose particle range holds the group is always opened.  A count
// pass, an exclusive scan and a fill pass make the CSR lists without
// atomics; ids come out in ascending order.
#include "nb_internal.h"

namespace nb {
namespace {

template <bool FILL>
__global__ void __launch_bounds__(256)
k_walk(int64_t n_groups, int64_t n_cell, const uint32_t* __restrict__ g_begin,
       const uint32_t* __restrict__ g_count, const double4* __restrict__ g_lo,
       const double4* __restrict__ g_hi, const uint4* __restrict__ meta,
       const double4* __restrict__ geo, uint32_t* __restrict__ cnt_e,
       uint32_t* __restrict__ cnt_s, const uint64_t* __restrict__ epj_off,
       const uint64_t* __restrict__ spj_off, uint32_t* __restrict__ epj,
       uint32_t* __restrict__ spj) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const uint32_t gb = g_begin[g];
  const uint32_t ge = gb + g_count[g];
  const double4 lo = g_lo[g], hi = g_hi[g];
  uint32_t* pe = nullptr;
  uint32_t* ps = nullptr;
  if (FILL) {
    pe = epj + epj_off[g];
    ps = spj + spj_off[g];
  }
  uint32_t ne = 0, ns = 0;
  uint32_t c = 0;
  const uint32_t nc = (uint32_t)n_cell;
  while (c < nc) {
    const uint4 m = meta[c];
    bool open;
    if (m.x <= gb && m.y >= ge) {
      open = true;
    } else {
      const double4 cc = geo[c];
      double dx = 0.0, dy = 0.0, dz = 0.0, t;
      t = __dsub_rn(lo.x, cc.x);
      if (t > dx) dx = t;
      t = __dsub_rn(cc.x, hi.x);
      if (t > dx) dx = t;
      t = __dsub_rn(lo.y, cc.y);
      if (t > dy) dy = t;
      t = __dsub_rn(cc.y, hi.y);
      if (t > dy) dy = t;
      t = __dsub_rn(lo.z, cc.z);
      if (t > dz) dz = t;
      t = __dsub_rn(cc.z, hi.z);
      if (t > dz) dz = t;
      const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                  __dmul_rn(dz, dz));
      open = !(d2 > cc.w);
    }
    // skip ids always point past the cell; the guard keeps a damaged tree
    // from looping forever
    const uint32_t next = (!open || ((m.w >> 8) & 1u)) ? m.z : c + 1;
    if (next <= c) break;
    if (!open) {
      if (FILL) ps[ns] = c;
      ++ns;
    } else if ((m.w >> 8) & 1u) {
      if (FILL)
        for (uint32_t j = m.x; j < m.y; ++j) pe[ne + (j - m.x)] = j;
      ne += m.y - m.x;
    }
    c = next;
  }
  if (!FILL) {
    cnt_e[g] = ne;
    cnt_s[g] = ns;
  }
}

// Interactions of the lists: sum over groups of n_i * (n_epj + n_spj).
__global__ void __launch_bounds__(256)
k_interactions(int64_t n_groups, const uint32_t* __restrict__ g_count,
               const uint32_t* __restrict__ cnt_e,
               const uint32_t* __restrict__ cnt_s,
               unsigned long long* __restrict__ out) {
  __shared__ unsigned long long s[4];
  unsigned long long v = 0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
       g < n_groups; g += (int64_t)gridDim.x * blockDim.x)
    v += (unsigned long long)g_count[g] *
         ((unsigned long long)cnt_e[g] + cnt_s[g]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, s[0] + s[1] + s[2] + s[3]);
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0ull;
}

}  // namespace

int launch_walk(nb_ctx* c, bool fill) {
  const size_t ng = (size_t)c->n_groups;
  int rc = reserve(c, c->cnt_e, ng);
  if (!rc) rc = reserve(c, c->cnt_s, ng);
  if (!rc) rc = reserve(c, c->epj_off, ng + 1);
  if (!rc) rc = reserve(c, c->spj_off, ng + 1);
  if (rc) return rc;
  auto k = fill ? k_walk<true> : k_walk<false>;
  hipLaunchKernelGGL(k, dim3(grid_for(c->n_groups, 256)), dim3(256), 0,
                     c->stream, c->n_groups, c->n_cell,
                     (const uint32_t*)c->g_begin.p,
                     (const uint32_t*)c->g_count.p, (const double4*)c->g_lo.p,
                     (const double4*)c->g_hi.p, (const uint4*)c->c_meta.p,
                     (const double4*)c->c_geo.p, c->cnt_e.p, c->cnt_s.p,
                     (const uint64_t*)c->epj_off.p,
                     (const uint64_t*)c->spj_off.p, c->epj.p, c->spj.p);
  return hip_check(c, hipGetLastError(), "walk launch");
}

// After the count pass: CSR offsets and the interaction count (red[0]).
int launch_list_stats(nb_ctx* c) {
  int rc = scan_u32_to_u64(c, c->cnt_e.p, c->epj_off.p, c->n_groups);
  if (!rc) rc = scan_u32_to_u64(c, c->cnt_s.p, c->spj_off.p, c->n_groups);
  if (!rc) rc = reserve(c, c->red, 8);
  if (rc) return rc;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, c->stream,
                     (unsigned long long*)c->red.p, 8);
  unsigned nb = grid_for(c->n_groups, 256);
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_interactions, dim3(nb), dim3(256), 0, c->stream,
                     c->n_groups, (const uint32_t*)c->g_count.p,
                     (const uint32_t*)c->cnt_e.p, (const uint32_t*)c->cnt_s.p,
                     (unsigned long long*)c->red.p);
  return hip_check(c, hipGetLastError(), "list stats launch");
}

}  // namespace nb
