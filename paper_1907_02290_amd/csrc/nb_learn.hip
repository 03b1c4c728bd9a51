// nb_learn.hip -- per-group list refresh and its learned predictor.  This
// extends the list reuse of section 4.2 (the paper keeps every list for a
// fixed number of steps): between two construction steps, the lists of
// single groups are walked again when a small perceptron predicts that
// their kept list has gone stale.
//
// Refresh mode (NB_FLAG_REFRESH) keeps per cell the FP64 centre of mass at
// construction and at the current step and the box of its current
// particles; in every opening test the cell's geometric centre is moved by
// the difference of the two centres of mass (a rigid motion changes no
// list), and its side becomes twice the largest distance from that centre
// to the particle box when that is larger (a cell whose particles spread is
// opened sooner).  Right after construction the shift is exactly zero, the
// side the geometric one, and the walk the plain one.  Per group it keeps the box, the cell shift and
// the opening-test slacks of the walk that made its list, and the list's
// age in reuse steps.  A kept list is stale at tolerance tau when one of its
// superparticles fails the opening test at angle theta (1 + tau): that is
// what the predictor learns to foresee without checking the list.
//
// Kernels: FP64 centres of mass (leaves, then levels bottom-up), shifted
// centres, predictor inputs, selection, the merge of refreshed and kept
// lists, and the 12-64-64-1 perceptron (forward; per-sample back-propagation;
// per-parameter sums over samples in fixed order; Adam).  The perceptron is
// 5057 parameters: one workgroup stages them in LDS and every lane runs one
// sample.  MFMA would need batches far larger than the group count to pay
// for the operand staging; at 131k groups a forward pass is ~1.3 GFLOP.
#include <cmath>
#include <cstring>
#include <mutex>
#include <utility>

#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kNF = NB_MLP_NIN;  // predictor inputs
constexpr int kNH = 64;          // hidden width
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kNH * kNF;
constexpr int kOffW2 = kOffB1 + kNH;
constexpr int kOffB2 = kOffW2 + kNH * kNH;
constexpr int kOffW3 = kOffB2 + kNH;
constexpr int kOffB3 = kOffW3 + kNH;
constexpr int kNP = kOffB3 + 1;
static_assert(kNP == NB_MLP_NPARAM, "parameter layout");
constexpr int kChunk = 1024;  // samples per partial gradient sum

__device__ inline uint32_t next_sibling(const CellRec* __restrict__ rec,
                                        uint32_t k, uint32_t stop) {
  const uint32_t s = rec[k].meta.z;
  return s > k ? s : stop;
}

// ---- FP64 centres of mass -------------------------------------------------
__global__ void __launch_bounds__(256)
k_com_leaf(int64_t cnt, const uint32_t* __restrict__ list,
           const CellRec* __restrict__ rec, const double4* __restrict__ pos,
           double4* __restrict__ com, double4* __restrict__ bmin,
           double4* __restrict__ bmax) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const uint32_t c = list[t];
  const uint4 m = rec[c].meta;
  const double4 g = rec[c].geo;
  double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
  double4 lo = pos[m.x], hi = lo;
  for (uint32_t p = m.x; p < m.y; ++p) {
    const double4 P = pos[p];
    M += P.w;
    sx += P.w * (P.x - g.x);
    sy += P.w * (P.y - g.y);
    sz += P.w * (P.z - g.z);
    lo.x = fmin(lo.x, P.x);
    lo.y = fmin(lo.y, P.y);
    lo.z = fmin(lo.z, P.z);
    hi.x = fmax(hi.x, P.x);
    hi.y = fmax(hi.y, P.y);
    hi.z = fmax(hi.z, P.z);
  }
  bmin[c] = lo;
  bmax[c] = hi;
  com[c] = M > 0.0 ? make_double4(g.x + sx / M, g.y + sy / M, g.z + sz / M, M)
                   : make_double4(g.x, g.y, g.z, 0.0);
}

__global__ void __launch_bounds__(256)
k_com_internal(int64_t cnt, const uint32_t* __restrict__ list,
               const CellRec* __restrict__ rec, double4* __restrict__ com,
               double4* __restrict__ bmin, double4* __restrict__ bmax) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const uint32_t c = list[t];
  const uint32_t stop = rec[c].meta.z;
  const double4 g = rec[c].geo;
  double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
  double4 lo = bmin[c + 1], hi = bmax[c + 1];
  for (uint32_t k = c + 1; k < stop; k = next_sibling(rec, k, stop)) {
    const double4 ck = com[k];
    M += ck.w;
    sx += ck.w * (ck.x - g.x);
    sy += ck.w * (ck.y - g.y);
    sz += ck.w * (ck.z - g.z);
    const double4 a = bmin[k], b = bmax[k];
    lo.x = fmin(lo.x, a.x);
    lo.y = fmin(lo.y, a.y);
    lo.z = fmin(lo.z, a.z);
    hi.x = fmax(hi.x, b.x);
    hi.y = fmax(hi.y, b.y);
    hi.z = fmax(hi.z, b.z);
  }
  bmin[c] = lo;
  bmax[c] = hi;
  com[c] = M > 0.0 ? make_double4(g.x + sx / M, g.y + sy / M, g.z + sz / M, M)
                   : make_double4(g.x, g.y, g.z, 0.0);
}

// Per cell: shift = com - com0, moved centre c' = geo + shift (rounded once
// each, as the FP64 reference does), and the side of the opening test: at a
// construction step (`fresh`) the geometric side s, so that construction
// walks are the plain opening test; later s, or twice the largest per-axis
// distance from c' to the box of the cell's current particles when that is
// larger.  (A particle can lie just outside its cube at construction: its
// key comes from the rounded x - lo.)  ctr.w = (side / theta)^2 -- at
// construction exactly the walk record's value, since s / theta =
// s (1 / theta) for a power of two s; shift.w = side.
__global__ void __launch_bounds__(256)
k_shift(int64_t nc, const CellRec* __restrict__ rec,
        const double4* __restrict__ com, const double4* __restrict__ com0,
        const double4* __restrict__ bmin, const double4* __restrict__ bmax,
        const Root* __restrict__ root, const uint32_t* __restrict__ seg,
        double theta, int fresh, double4* __restrict__ shift,
        double4* __restrict__ ctr) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double4 a = com[c], b = com0[c], g = rec[c].geo;
  const uint4 m = rec[c].meta;
  const double sx = __dsub_rn(a.x, b.x), sy = __dsub_rn(a.y, b.y),
               sz = __dsub_rn(a.z, b.z);
  const double cx = __dadd_rn(g.x, sx), cy = __dadd_rn(g.y, sy),
               cz = __dadd_rn(g.z, sz);
  const double4 lo = bmin[c], hi = bmax[c];
  double h = 0.0;
  h = fmax(h, __dsub_rn(hi.x, cx));
  h = fmax(h, __dsub_rn(cx, lo.x));
  h = fmax(h, __dsub_rn(hi.y, cy));
  h = fmax(h, __dsub_rn(cy, lo.y));
  h = fmax(h, __dsub_rn(hi.z, cz));
  h = fmax(h, __dsub_rn(cz, lo.z));
  const double s = ldexp(1.0, root[seg[m.x]].k - (int)(m.w & 255u));
  const double w = 2.0 * h;
  const double side = (!fresh && w > s) ? w : s;
  const double r = __ddiv_rn(side, theta);
  shift[c] = make_double4(sx, sy, sz, side);
  ctr[c] = make_double4(cx, cy, cz, __dmul_rn(r, r));
}

__global__ void __launch_bounds__(256)
k_age_inc(int64_t ng, uint32_t* __restrict__ age) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ng && age[g] < 0xFFFFFFFFu) age[g] += 1u;
}

// ---- predictor inputs -------------------------------------------------------
__device__ inline double capped(double a, double b) {
  const double cap = 1e6;
  if (b > 0.0) {
    const double q = a / b;
    return q < cap ? q : cap;
  }
  return a > 0.0 ? cap : 0.0;
}

__global__ void __launch_bounds__(256)
k_features(int64_t ng, const uint32_t* __restrict__ g_cell,
           const uint32_t* __restrict__ g_begin,
           const uint32_t* __restrict__ g_count,
           const CellRec* __restrict__ rec, const Root* __restrict__ root,
           const uint32_t* __restrict__ seg, const double4* __restrict__ clo,
           const double4* __restrict__ chi, const double4* __restrict__ lo0,
           const double4* __restrict__ hi0,
           const double4* __restrict__ tau0,
           const double4* __restrict__ shift, const double* __restrict__ g_sa,
           const double* __restrict__ g_so, const uint32_t* __restrict__ age,
           const uint32_t* __restrict__ cnt_e,
           const uint32_t* __restrict__ cnt_s, int kmax,
           float* __restrict__ feat) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const uint32_t c = g_cell[g];
  const int level = (int)(rec[c].meta.w & 255u);
  const int k = root[seg[g_begin[g]]].k;
  const double s = ldexp(1.0, k - level);
  const double4 lo = clo[g], hi = chi[g], a0 = lo0[g], b0 = hi0[g];
  const double4 t0 = tau0[g], sh = shift[c];
  const double dt[3] = {sh.x - t0.x, sh.y - t0.y, sh.z - t0.z};
  const double l[3] = {lo.x, lo.y, lo.z}, h[3] = {hi.x, hi.y, hi.z};
  const double l0[3] = {a0.x, a0.y, a0.z}, h0[3] = {b0.x, b0.y, b0.z};
  double e[3], grow = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double dl = fabs((l[a] - l0[a]) - dt[a]);
    const double dh = fabs((h[a] - h0[a]) - dt[a]);
    e[a] = dl > dh ? dl : dh;
    const double w = (h[a] - l[a]) - (h0[a] - l0[a]);
    if (w > grow) grow = w;
  }
  const double E = sqrt((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]);
  const double B = sqrt((dt[0] * dt[0] + dt[1] * dt[1]) + dt[2] * dt[2]);
  const double sa = g_sa[g], so = g_so[g];
  const double nl = (double)cnt_e[g] + (double)cnt_s[g];
  const uint32_t ag = age[g];
  float* f = feat + (int64_t)kNF * g;
  f[0] = (float)((double)(ag < (uint32_t)kmax ? ag : (uint32_t)kmax) / kmax);
  f[1] = (float)log1p(capped(E, sa));
  f[2] = (float)log1p(capped(E, so));
  f[3] = (float)log1p(capped(B, sa));
  f[4] = (float)log1p(capped(B, so));
  f[5] = (float)log1p(E / s);
  f[6] = (float)log1p(B / s);
  f[7] = (float)log1p(capped(sa, s));
  f[8] = (float)log1p(capped(so, s));
  f[9] = (float)log1p(grow / s);
  f[10] = (float)(log2((double)g_count[g]) / 6.0);
  f[11] = (float)(log2(1.0 + nl) / 16.0);
}

// ---- staleness labels -------------------------------------------------------
// A kept list is stale when one of its superparticles fails the opening
// test at the relaxed angle theta' = theta (1 + tau) from the group's current
// box and the cell's current centre and side: (side / theta')^2.
// One wave per group: the lanes test 64 kept superparticles at a time and a
// ballot ends the group at the first failing stretch.
__global__ void __launch_bounds__(256)
k_check_lists(int64_t ng, const double4* __restrict__ clo,
              const double4* __restrict__ chi,
              const double4* __restrict__ ctr,
              const double4* __restrict__ shift,
              const uint64_t* __restrict__ spj_off,
              const uint32_t* __restrict__ cnt_s,
              const uint32_t* __restrict__ spj, double th,
              uint8_t* __restrict__ stale) {
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= ng) return;
  const double4 lo = clo[g], hi = chi[g];
  bool bad = false;
  for (uint64_t j0 = spj_off[g], e = j0 + cnt_s[g]; j0 < e; j0 += 64) {
    const uint64_t j = j0 + lane;
    bool b = false;
    if (j < e) {
      const uint32_t c = spj[j];
      const double4 cc = ctr[c];
      const double r = __ddiv_rn(shift[c].w, th);
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
      const double d2 = __dadd_rn(
          __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
      b = !(d2 > __dmul_rn(r, r));
    }
    if (__ballot(b)) {
      bad = true;
      break;
    }
  }
  if (lane == 0) stale[g] = (uint8_t)bad;
}

// ---- selection and list merge ----------------------------------------------
__global__ void __launch_bounds__(256)
k_select(int64_t ng, const float* __restrict__ prob,
         const uint32_t* __restrict__ age, float p_star, uint32_t kmax,
         uint32_t* __restrict__ pick) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ng) pick[g] = (prob[g] > p_star || age[g] >= kmax) ? 1u : 0u;
}

__global__ void __launch_bounds__(256)
k_select_stale(int64_t ng, const uint8_t* __restrict__ stale,
               const uint32_t* __restrict__ age, uint32_t kmax,
               uint32_t* __restrict__ pick) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ng) pick[g] = (stale[g] || age[g] >= kmax) ? 1u : 0u;
}

__global__ void __launch_bounds__(256)
k_mark(int64_t n_sel, const uint32_t* __restrict__ sel,
       uint32_t* __restrict__ pick) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_sel) pick[sel[t]] = 1u;
}

__global__ void __launch_bounds__(256)
k_compact(int64_t ng, const uint32_t* __restrict__ pick,
          const uint32_t* __restrict__ pos, uint32_t* __restrict__ sel) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ng && pick[g]) sel[pos[g]] = (uint32_t)g;
}

// A refreshed list replaces the kept one only where it fits: the tokens of
// each walk lane in the lane's room (lane_off, by group), its particle and
// superparticle ids in the group's list slot (the slots' offsets are CSR,
// so a slot ends where the next begins).  Counts the refreshed groups and
// those left as they were.
__global__ void __launch_bounds__(256)
k_refresh_fit(int64_t n_max, const uint32_t* __restrict__ n_dev,
              const uint32_t* __restrict__ sel,
              const uint32_t* __restrict__ sel_e,
              const uint32_t* __restrict__ sel_s,
              const uint32_t* __restrict__ sel_tl,
              const uint64_t* __restrict__ lane_off,
              const uint64_t* __restrict__ epj_off,
              const uint64_t* __restrict__ spj_off,
              uint8_t* __restrict__ ok, unsigned long long* __restrict__ red) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_max || t >= (int64_t)*n_dev) return;
  const uint32_t g = sel[t];
  bool fits = (uint64_t)sel_e[t] <= epj_off[g + 1] - epj_off[g] &&
              (uint64_t)sel_s[t] <= spj_off[g + 1] - spj_off[g];
  for (int h = 0; h < kSplitLanes; ++h) {
    const uint64_t* r = lane_off + (uint64_t)g * kSplitLanes + h;
    fits = fits && (uint64_t)sel_tl[(uint64_t)t * kSplitLanes + h] <= r[1] - r[0];
  }
  ok[t] = fits ? 1 : 0;
  atomicAdd(red + (fits ? kRedRefreshed : kRedOverflow), 1ull);
}

// Install what fitted: lengths, the walk's slacks and cell shift, the box the
// list was walked for, age 0.  A group that did not fit keeps its list and
// state (and stays due: its age keeps growing).
__global__ void __launch_bounds__(256)
k_refresh_commit(int64_t n_max, const uint32_t* __restrict__ n_dev,
                 const uint32_t* __restrict__ sel,
                 const uint8_t* __restrict__ ok,
                 const uint32_t* __restrict__ sel_e,
                 const uint32_t* __restrict__ sel_s,
                 const double* __restrict__ sel_sa,
                 const double* __restrict__ sel_so,
                 const double4* __restrict__ sel_tau0,
                 const double4* __restrict__ clo,
                 const double4* __restrict__ chi,
                 uint32_t* __restrict__ cnt_e, uint32_t* __restrict__ cnt_s,
                 double* __restrict__ g_sa, double* __restrict__ g_so,
                 double4* __restrict__ g_tau0, double4* __restrict__ lo,
                 double4* __restrict__ hi, uint32_t* __restrict__ age) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_max || t >= (int64_t)*n_dev || !ok[t]) return;
  const uint32_t g = sel[t];
  cnt_e[g] = sel_e[t];
  cnt_s[g] = sel_s[t];
  g_sa[g] = sel_sa[t];
  g_so[g] = sel_so[t];
  g_tau0[g] = sel_tau0[t];
  lo[g] = clo[g];
  hi[g] = chi[g];
  age[g] = 0u;
}

// Slot and lane-room sizes after a refresh some of whose lists did not fit:
// every group keeps its slot's and its lanes' sizes (k_slot_sizes), a group
// whose walked list did not fit gets twice that list plus 32 entries, and
// each of its lanes twice the lane's tokens plus kLaneSpare (k_slot_grow).
__global__ void __launch_bounds__(256)
k_slot_sizes(int64_t ng, const uint64_t* __restrict__ epj_off,
             const uint64_t* __restrict__ spj_off,
             const uint64_t* __restrict__ lane_off,
             uint32_t* __restrict__ cap_e, uint32_t* __restrict__ cap_s,
             uint32_t* __restrict__ lane_cap) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  cap_e[g] = (uint32_t)(epj_off[g + 1] - epj_off[g]);
  cap_s[g] = (uint32_t)(spj_off[g + 1] - spj_off[g]);
  for (int h = 0; h < kSplitLanes; ++h) {
    const uint64_t i = (uint64_t)g * kSplitLanes + h;
    lane_cap[i] = (uint32_t)(lane_off[i + 1] - lane_off[i]);
  }
}

__global__ void __launch_bounds__(256)
k_slot_grow(int64_t n_max, const uint32_t* __restrict__ n_dev,
            const uint32_t* __restrict__ sel, const uint8_t* __restrict__ ok,
            const uint32_t* __restrict__ sel_e,
            const uint32_t* __restrict__ sel_s,
            const uint32_t* __restrict__ sel_tl, uint32_t* __restrict__ cap_e,
            uint32_t* __restrict__ cap_s, uint32_t* __restrict__ lane_cap) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_max || t >= (int64_t)*n_dev || ok[t]) return;
  const uint32_t g = sel[t];
  const uint32_t e = 2u * sel_e[t] + 32u, s = 2u * sel_s[t] + 32u;
  if (e > cap_e[g]) cap_e[g] = e;
  if (s > cap_s[g]) cap_s[g] = s;
  for (int h = 0; h < kSplitLanes; ++h) {
    const uint64_t i = (uint64_t)g * kSplitLanes + h;
    const uint32_t r =
        (2u * sel_tl[(uint64_t)t * kSplitLanes + h] + kLaneSpare + 15u) & ~15u;
    if (r > lane_cap[i]) lane_cap[i] = r;
  }
}

// Every group's list from its old slot to its new one (one wave per group).
__global__ void __launch_bounds__(256)
k_slot_move(int64_t ng, const uint32_t* __restrict__ cnt_e,
            const uint32_t* __restrict__ cnt_s,
            const uint64_t* __restrict__ eo, const uint32_t* __restrict__ e,
            const uint64_t* __restrict__ so, const uint32_t* __restrict__ s,
            const uint64_t* __restrict__ eo2, uint32_t* __restrict__ e2,
            const uint64_t* __restrict__ so2, uint32_t* __restrict__ s2) {
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= ng) return;
  const uint64_t a = eo[g], a2 = eo2[g], na = cnt_e[g];
  for (uint64_t i = lane; i < na; i += 64) e2[a2 + i] = e[a + i];
  const uint64_t b = so[g], b2 = so2[g], nb = cnt_s[g];
  for (uint64_t i = lane; i < nb; i += 64) s2[b2 + i] = s[b + i];
}

__global__ void k_zero_u64s(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void __launch_bounds__(256)
k_u8_to_f32(int64_t n, const uint8_t* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ---- perceptron ---------------------------------------------------------------
__device__ inline void stage_weights(const float* __restrict__ w, float* sw) {
  for (int q = threadIdx.x; q < kNP; q += blockDim.x) sw[q] = w[q];
  __syncthreads();
}

// log(1 + exp(z)) without overflow
__device__ inline float softplus(float z) {
  return z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));
}

__device__ inline float forward_one(const float* sw, const float* __restrict__ xr,
                                    float* h1, float* h2) {
  float xi[kNF];
#pragma unroll
  for (int k = 0; k < kNF; ++k) xi[k] = xr[k];
#pragma unroll
  for (int j = 0; j < kNH; ++j) {
    float s = sw[kOffB1 + j];
#pragma unroll
    for (int k = 0; k < kNF; ++k) s = fmaf(sw[kOffW1 + j * kNF + k], xi[k], s);
    h1[j] = tanhf(s);
  }
  float z = sw[kOffB3];
#pragma unroll
  for (int j = 0; j < kNH; ++j) {
    float s = sw[kOffB2 + j];
#pragma unroll
    for (int k = 0; k < kNH; ++k) s = fmaf(sw[kOffW2 + j * kNH + k], h1[k], s);
    h2[j] = tanhf(s);
    z = fmaf(sw[kOffW3 + j], h2[j], z);
  }
  return z;
}

__global__ void __launch_bounds__(256)
k_mlp_fwd(int64_t n, const float* __restrict__ x, const float* __restrict__ w,
          float* __restrict__ p) {
  __shared__ float sw[kNP];
  stage_weights(w, sw);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float h1[kNH], h2[kNH];
  const float z = forward_one(sw, x + (int64_t)kNF * i, h1, h2);
  p[i] = 1.f / (1.f + expf(-z));
}

// Per sample: loss term, output delta dz = dL/dz, hidden deltas and the
// activations the parameter sums need (rows of 64 floats per sample).
__global__ void __launch_bounds__(256)
k_mlp_bwd(int64_t n, const float* __restrict__ x, const float* __restrict__ y,
          const float* __restrict__ w, float pw, float inv_n,
          float* __restrict__ H1, float* __restrict__ H2,
          float* __restrict__ D1, float* __restrict__ D2,
          float* __restrict__ DZ, float* __restrict__ lossp) {
  __shared__ float sw[kNP];
  __shared__ float red[4];
  stage_weights(w, sw);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float li = 0.f;
  if (i < n) {
    float h1[kNH], h2[kNH];
    const float z = forward_one(sw, x + (int64_t)kNF * i, h1, h2);
    const float p = 1.f / (1.f + expf(-z));
    const float yi = y[i];
    const float wy = pw * yi;
    li = wy * softplus(-z) + (1.f - yi) * softplus(z);
    const float dz = (p * (wy + 1.f - yi) - wy) * inv_n;
    DZ[i] = dz;
    float* h1r = H1 + (int64_t)kNH * i;
    float* h2r = H2 + (int64_t)kNH * i;
    float* d2r = D2 + (int64_t)kNH * i;
    float* d1r = D1 + (int64_t)kNH * i;
    float d2[kNH];
#pragma unroll
    for (int j = 0; j < kNH; ++j) {
      d2[j] = dz * sw[kOffW3 + j] * (1.f - h2[j] * h2[j]);
      h1r[j] = h1[j];
      h2r[j] = h2[j];
      d2r[j] = d2[j];
    }
#pragma unroll
    for (int k = 0; k < kNH; ++k) {
      float s = 0.f;
#pragma unroll
      for (int j = 0; j < kNH; ++j) s = fmaf(d2[j], sw[kOffW2 + j * kNH + k], s);
      d1r[k] = s * (1.f - h1[k] * h1[k]);
    }
  }
  // block sum of the loss terms, fixed order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) li += __shfl_xor(li, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = li;
  __syncthreads();
  if (threadIdx.x == 0) lossp[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Partial gradient of every parameter over one chunk of samples
// (blockIdx.y), summed in sample order.
__global__ void __launch_bounds__(256)
k_mlp_wgrad(int64_t n, const float* __restrict__ x,
            const float* __restrict__ H1, const float* __restrict__ H2,
            const float* __restrict__ D1, const float* __restrict__ D2,
            const float* __restrict__ DZ, float* __restrict__ part) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kNP) return;
  const int64_t b0 = (int64_t)blockIdx.y * kChunk;
  const int64_t b1 = b0 + kChunk < n ? b0 + kChunk : n;
  float s = 0.f;
  if (q < kOffB1) {
    const int j = q / kNF, k = q % kNF;
    for (int64_t b = b0; b < b1; ++b)
      s = fmaf(D1[b * kNH + j], x[b * kNF + k], s);
  } else if (q < kOffW2) {
    const int j = q - kOffB1;
    for (int64_t b = b0; b < b1; ++b) s += D1[b * kNH + j];
  } else if (q < kOffB2) {
    const int r = q - kOffW2, j = r / kNH, k = r % kNH;
    for (int64_t b = b0; b < b1; ++b)
      s = fmaf(D2[b * kNH + j], H1[b * kNH + k], s);
  } else if (q < kOffW3) {
    const int j = q - kOffB2;
    for (int64_t b = b0; b < b1; ++b) s += D2[b * kNH + j];
  } else if (q < kOffB3) {
    const int k = q - kOffW3;
    for (int64_t b = b0; b < b1; ++b) s = fmaf(DZ[b], H2[b * kNH + k], s);
  } else {
    for (int64_t b = b0; b < b1; ++b) s += DZ[b];
  }
  part[(int64_t)blockIdx.y * kNP + q] = s;
}

__global__ void __launch_bounds__(256)
k_mlp_reduce(int n_chunks, const float* __restrict__ part,
             float* __restrict__ grad, int n_lossp,
             const float* __restrict__ lossp, float inv_n,
             float* __restrict__ loss) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < kNP) {
    float s = 0.f;
    for (int c = 0; c < n_chunks; ++c) s += part[(int64_t)c * kNP + q];
    grad[q] = s;
  }
  if (q == 0) {
    float s = 0.f;
    for (int b = 0; b < n_lossp; ++b) s += lossp[b];
    *loss = s * inv_n;
  }
}

__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ w, const float* __restrict__ g,
       float* __restrict__ m, float* __restrict__ v, float lr, float b1,
       float b2, float eps, float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kNP) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

}  // namespace

// ---- launchers ----------------------------------------------------------------

int learn_reserve_cells(nb_ctx* c) {
  const size_t nc = (size_t)c->n_cell;
  int rc = reserve(c, c->c_com, nc);
  if (!rc) rc = reserve(c, c->c_com0, nc);
  if (!rc) rc = reserve(c, c->c_bmin, nc);
  if (!rc) rc = reserve(c, c->c_bmax, nc);
  if (!rc) rc = reserve(c, c->c_shift, nc);
  if (!rc) rc = reserve(c, c->c_ctr, nc);
  return rc;
}

int learn_reserve_groups(nb_ctx* c) {
  const size_t ng = (size_t)c->n_groups;
  int rc = reserve(c, c->g_clo, ng);
  if (!rc) rc = reserve(c, c->g_chi, ng);
  if (!rc) rc = reserve(c, c->g_tau0, ng);
  if (!rc) rc = reserve(c, c->g_sa, ng);
  if (!rc) rc = reserve(c, c->g_so, ng);
  if (!rc) rc = reserve(c, c->g_age, ng);
  if (!rc) rc = reserve(c, c->pick, ng + 1);
  if (!rc) rc = reserve(c, c->pickpos, ng + 1);
  if (!rc) rc = reserve(c, c->sel, ng);
  if (!rc) rc = reserve(c, c->ne2, ng);
  if (!rc) rc = reserve(c, c->ns2, ng);
  if (!rc) rc = reserve(c, c->feat, (size_t)kNF * ng);
  if (!rc) rc = reserve(c, c->prob, ng);
  if (!rc) rc = reserve(c, c->stale, ng);
  if (!rc) rc = reserve(c, c->sel_e, ng);
  if (!rc) rc = reserve(c, c->sel_s, ng);
  if (!rc) rc = reserve(c, c->sel_t, ng);
  if (!rc) rc = reserve(c, c->sel_sa, ng);
  if (!rc) rc = reserve(c, c->sel_so, ng);
  if (!rc) rc = reserve(c, c->sel_tau0, ng);
  if (!rc) rc = reserve(c, c->sel_ok, ng);
  return rc;
}

// Centres of mass in FP64 and the shifted centres.  At a construction step
// (c->in_build) the construction-time centres are set to the current ones
// first, so every shift is zero.
int launch_com(nb_ctx* c) {
  int rc = learn_reserve_cells(c);
  if (rc) return rc;
  if (c->n_leaves > 0)
    hipLaunchKernelGGL(k_com_leaf, dim3(grid_for(c->n_leaves, 256)),
                       dim3(256), 0, c->stream, c->n_leaves,
                       (const uint32_t*)c->lvl_cells.p + c->lvl_off[kLevels],
                       (const CellRec*)c->c_rec.p, (const double4*)c->pos.p,
                       c->c_com.p, c->c_bmin.p, c->c_bmax.p);
  for (int l = kMaxLevel - 1; l >= 0; --l) {
    const int64_t cnt = c->lvl_count[l];
    if (cnt == 0) continue;
    hipLaunchKernelGGL(k_com_internal, dim3(grid_for(cnt, 256)), dim3(256), 0,
                       c->stream, cnt,
                       (const uint32_t*)c->lvl_cells.p + c->lvl_off[l],
                       (const CellRec*)c->c_rec.p, c->c_com.p, c->c_bmin.p,
                       c->c_bmax.p);
  }
  rc = hip_check(c, hipGetLastError(), "centre-of-mass launch");
  if (rc) return rc;
  if (c->in_build) {
    rc = hip_check(c, hipMemcpyAsync(c->c_com0.p, c->c_com.p,
                                     (size_t)c->n_cell * sizeof(double4),
                                     hipMemcpyDeviceToDevice, c->stream),
                   "centre-of-mass copy");
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_shift, dim3(grid_for(c->n_cell, 256)), dim3(256), 0,
                     c->stream, c->n_cell, (const CellRec*)c->c_rec.p,
                     (const double4*)c->c_com.p, (const double4*)c->c_com0.p,
                     (const double4*)c->c_bmin.p, (const double4*)c->c_bmax.p,
                     (const Root*)c->root.p, (const uint32_t*)c->seg.p,
                     c->cfg.theta, c->in_build ? 1 : 0, c->c_shift.p,
                     c->c_ctr.p);
  return hip_check(c, hipGetLastError(), "shift launch");
}

int learn_after_groups(nb_ctx* c) {
  int rc = learn_reserve_groups(c);
  if (!rc) rc = fill_u32(c, c->g_age.p, c->n_groups, 0u);
  return rc;
}

int launch_age_inc(nb_ctx* c) {
  hipLaunchKernelGGL(k_age_inc, dim3(grid_for(c->n_groups, 256)), dim3(256),
                     0, c->stream, c->n_groups, c->g_age.p);
  return hip_check(c, hipGetLastError(), "age launch");
}

int launch_features(nb_ctx* c) {
  int rc = launch_group_box(c, c->g_clo.p, c->g_chi.p);
  if (rc) return rc;
  hipLaunchKernelGGL(k_features, dim3(grid_for(c->n_groups, 256)), dim3(256),
                     0, c->stream, c->n_groups, (const uint32_t*)c->g_cell.p,
                     (const uint32_t*)c->g_begin.p,
                     (const uint32_t*)c->g_count.p, (const CellRec*)c->c_rec.p,
                     (const Root*)c->root.p, (const uint32_t*)c->seg.p,
                     (const double4*)c->g_clo.p, (const double4*)c->g_chi.p,
                     (const double4*)c->g_lo.p, (const double4*)c->g_hi.p,
                     (const double4*)c->g_tau0.p,
                     (const double4*)c->c_shift.p, (const double*)c->g_sa.p,
                     (const double*)c->g_so.p, (const uint32_t*)c->g_age.p,
                     (const uint32_t*)c->cnt_e.p,
                     (const uint32_t*)c->cnt_s.p, c->cfg.k_max, c->feat.p);
  return hip_check(c, hipGetLastError(), "feature launch");
}

int launch_stale(nb_ctx* c, double tau) {
  int rc = launch_group_box(c, c->g_clo.p, c->g_chi.p);
  if (rc) return rc;
  const double th = c->cfg.theta * (1.0 + tau);
  hipLaunchKernelGGL(k_check_lists, dim3(grid_for(c->n_groups, 4)),
                     dim3(256), 0, c->stream, c->n_groups,
                     (const double4*)c->g_clo.p, (const double4*)c->g_chi.p,
                     (const double4*)c->c_ctr.p, (const double4*)c->c_shift.p,
                     (const uint64_t*)c->spj_off.p,
                     (const uint32_t*)c->cnt_s.p, (const uint32_t*)c->spj.p,
                     th, c->stale.p);
  return hip_check(c, hipGetLastError(), "list check launch");
}

int mlp_forward(nb_ctx* c, int64_t n, const float* x, float* p) {
  if (n <= 0) return NB_OK;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(grid_for(n, 256)), dim3(256), 0,
                     c->stream, n, x, (const float*)c->mlp_w.p, p);
  return hip_check(c, hipGetLastError(), "perceptron launch");
}

// Gradient of the mean (weighted) cross-entropy over samples [0, n) of x, y
// into grad[0, NP) and the loss into *loss (device), with the per-sample
// activations and deltas in act (4 kNH n floats), the output deltas in dz
// (n), the per-block loss terms in lossp (ceil(n / 256)) and the per-chunk
// partial sums in part (ceil(n / kChunk) kNP).  Every scratch value read is
// written earlier in the same call, so none needs clearing.
static int mlp_grad_into(nb_ctx* c, int64_t n, const float* x, const float* y,
                         float pw, float* act, float* dz, float* lossp,
                         float* part, float* grad, float* loss) {
  const int64_t nlp = grid_for(n, 256);
  const int64_t nch = (n + kChunk - 1) / kChunk;
  float* H1 = act;
  float* H2 = H1 + (size_t)kNH * n;
  float* D1 = H2 + (size_t)kNH * n;
  float* D2 = D1 + (size_t)kNH * n;
  const float inv_n = (float)(1.0 / (double)n);
  hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)nlp), dim3(256), 0, c->stream,
                     n, x, y, (const float*)c->mlp_w.p, pw, inv_n, H1, H2, D1,
                     D2, dz, lossp);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(grid_for(kNP, 256), (unsigned)nch),
                     dim3(256), 0, c->stream, n, x, (const float*)H1,
                     (const float*)H2, (const float*)D1, (const float*)D2,
                     (const float*)dz, part);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(grid_for(kNP, 256)), dim3(256), 0,
                     c->stream, (int)nch, (const float*)part, grad, (int)nlp,
                     (const float*)lossp, inv_n, loss);
  return hip_check(c, hipGetLastError(), "perceptron gradient launch");
}

// The same into c->mlp_g[0, NP) and the loss into c->mlp_g[NP], with scratch
// the context allocates (and keeps) for n samples.
int mlp_grad(nb_ctx* c, int64_t n, const float* x, const float* y, float pw) {
  const int64_t nlp = grid_for(n, 256);
  const int64_t nch = (n + kChunk - 1) / kChunk;
  int rc = reserve(c, c->mlp_act, (size_t)4 * kNH * n);
  if (!rc) rc = reserve(c, c->mlp_dz, (size_t)n);
  if (!rc) rc = reserve(c, c->mlp_lossp, (size_t)nlp);
  if (!rc) rc = reserve(c, c->mlp_part, (size_t)nch * kNP);
  if (rc) return rc;
  return mlp_grad_into(c, n, x, y, pw, c->mlp_act.p, c->mlp_dz.p,
                       c->mlp_lossp.p, c->mlp_part.p, c->mlp_g.p,
                       c->mlp_g.p + kNP);
}

// ---- the allocation-free gradient (nb_mlp_grad_static) -----------------------
// Its scratch is this file-scope array: one copy per GPU, held until the
// process ends, shared by every context and call on that GPU.  Layout in
// floats, each part starting on a 256-byte boundary: activations and deltas
// (4 kNH rows), output deltas (rows), per-block loss terms (rows / 256),
// per-chunk partial gradients (rows / kChunk x kNP), and a loss slot used
// when the caller passes no loss pointer.
constexpr int64_t kStaticRows = NB_MLP_STATIC_MAX_ROWS;
static_assert(kStaticRows % kChunk == 0 && kStaticRows % 256 == 0,
              "static scratch rows");
constexpr size_t align64(size_t v) { return (v + 63) / 64 * 64; }
constexpr size_t kSAct = 0;
constexpr size_t kSDz = kSAct + align64((size_t)4 * kNH * kStaticRows);
constexpr size_t kSLoss = kSDz + align64((size_t)kStaticRows);
constexpr size_t kSPart = kSLoss + align64((size_t)kStaticRows / 256);
constexpr size_t kSSink =
    kSPart + align64((size_t)(kStaticRows / kChunk) * kNP);
constexpr size_t kScratchFloats = kSSink + 64;

static __device__ __align__(256) float scratch[kScratchFloats];

// Device address of `scratch` on each GPU (the host-side name is only a
// stand-in: a kernel given it would fault).  Looked up once per device.
constexpr int kMaxDevices = 64;
static float* g_scratch_dev[kMaxDevices] = {};

int static_scratch_init(nb_ctx* c) {
  static std::mutex mu;
  if (c->device < 0 || c->device >= kMaxDevices)
    return set_err(c, NB_ERR_HIP, "device %d beyond the static scratch table",
                   c->device);
  std::lock_guard<std::mutex> lock(mu);
  if (g_scratch_dev[c->device]) return NB_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return set_err(c, NB_ERR_HIP, "hipGetSymbolAddress(scratch): %s",
                   hipGetErrorString(e));
  }
  g_scratch_dev[c->device] = static_cast<float*>(ptr);
  return NB_OK;
}

int mlp_adam(nb_ctx* c, const float* g, float lr, float b1, float b2,
             float eps) {
  c->mlp_t += 1;
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)c->mlp_t));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)c->mlp_t));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(kNP, 256)), dim3(256), 0,
                     c->stream, c->mlp_w.p, g, c->mlp_m.p, c->mlp_v.p, lr, b1,
                     b2, eps, c1, c2);
  return hip_check(c, hipGetLastError(), "adam launch");
}

int mlp_ensure(nb_ctx* c) {
  if (c->mlp_w.p) return NB_OK;
  int rc = reserve(c, c->mlp_w, kNP);
  if (!rc) rc = reserve(c, c->mlp_m, kNP);
  if (!rc) rc = reserve(c, c->mlp_v, kNP);
  if (!rc) rc = reserve(c, c->mlp_g, kNP + 1);
  if (rc) return rc;
  // zero weights: p = 1/2 everywhere
  rc = hip_check(c, hipMemsetAsync(c->mlp_w.p, 0, kNP * 4, c->stream), "init");
  if (!rc) rc = hip_check(c, hipMemsetAsync(c->mlp_m.p, 0, kNP * 4, c->stream), "init");
  if (!rc) rc = hip_check(c, hipMemsetAsync(c->mlp_v.p, 0, kNP * 4, c->stream), "init");
  c->mlp_t = 0;
  return rc;
}

// Refresh the lists of the groups flagged in c->pick (their ids compacted
// into c->sel in ascending order, their number at c->pickpos[n_groups] on
// the device), without waiting for the host: one walk pass over up to all
// groups' slots (the kernels read the selection size), kSplitLanes lanes
// per group, each lane's tokens into its group's lane room; then each
// refreshed list that fits its lanes' room and its group's list slot is
// expanded into the slot and installed (k_refresh_fit / k_expand /
// k_refresh_commit), the others keep their lists; last, the interaction
// counts of the current lists (device counters).  The current boxes must be
// in g_clo / g_chi.  Every buffer was sized by the construction step, so a
// refresh allocates nothing and can be captured in a HIP graph.
int refresh_selected(nb_ctx* c) {
  const int64_t G = c->n_groups;
  const uint32_t* n_dev = c->pickpos.p + G;
  if (!c->red.p || !c->lane_off.p ||
      (uint64_t)c->lane_total > c->tok.cap ||
      (uint64_t)G * kSplitLanes > c->cnt_tl.cap)
    return set_err(c, NB_ERR_STATE, "refresh buffers not sized");
  const WalkOut o{c->sel_e.p, c->sel_s.p, c->sel_t.p, c->sel_sa.p,
                  c->sel_so.p, c->sel_tau0.p, n_dev};
  int rc = launch_walk_refresh(c, G, c->sel.p, c->g_clo.p, c->g_chi.p, o);
  if (rc) return rc;
  unsigned long long* red = reinterpret_cast<unsigned long long*>(c->red.p);
  hipLaunchKernelGGL(k_zero_u64s, dim3(1), dim3(64), 0, c->stream,
                     red + kRedRefreshed, 2);
  hipLaunchKernelGGL(k_refresh_fit, dim3(grid_for(G, 256)), dim3(256), 0,
                     c->stream, G, n_dev, (const uint32_t*)c->sel.p,
                     (const uint32_t*)c->sel_e.p, (const uint32_t*)c->sel_s.p,
                     (const uint32_t*)c->cnt_tl.p,
                     (const uint64_t*)c->lane_off.p,
                     (const uint64_t*)c->epj_off.p,
                     (const uint64_t*)c->spj_off.p, c->sel_ok.p, red);
  rc = hip_check(c, hipGetLastError(), "refresh fit launch");
  if (!rc) rc = launch_expand_sel(c, G, c->sel.p, n_dev, c->sel_ok.p);
  if (rc) return rc;
  hipLaunchKernelGGL(k_refresh_commit, dim3(grid_for(G, 256)), dim3(256), 0,
                     c->stream, G, n_dev, (const uint32_t*)c->sel.p,
                     (const uint8_t*)c->sel_ok.p, (const uint32_t*)c->sel_e.p,
                     (const uint32_t*)c->sel_s.p, (const double*)c->sel_sa.p,
                     (const double*)c->sel_so.p,
                     (const double4*)c->sel_tau0.p, (const double4*)c->g_clo.p,
                     (const double4*)c->g_chi.p, c->cnt_e.p, c->cnt_s.p,
                     c->g_sa.p, c->g_so.p, c->g_tau0.p, c->g_lo.p, c->g_hi.p,
                     c->g_age.p);
  rc = hip_check(c, hipGetLastError(), "refresh commit launch");
  if (!rc) rc = launch_interactions(c, c->cnt_e.p, c->cnt_s.p);
  return rc;
}

// After a refresh whose lists did not all fit (the selection and its walk's
// output are still in place): larger list slots and lane rooms for those
// groups, every list moved to its new slot, and the token buffer grown to
// the new rooms.  Synchronises with the host.  Drops a captured graph (the
// list buffers change).
static int grow_slots(nb_ctx* c) {
  const int64_t G = c->n_groups;
  const int64_t nl = (int64_t)kSplitLanes * G;
  const uint32_t* n_dev = c->pickpos.p + G;
  hipLaunchKernelGGL(k_slot_sizes, dim3(grid_for(G, 256)), dim3(256), 0,
                     c->stream, G, (const uint64_t*)c->epj_off.p,
                     (const uint64_t*)c->spj_off.p,
                     (const uint64_t*)c->lane_off.p, c->ne2.p, c->ns2.p,
                     c->lane_cap.p);
  hipLaunchKernelGGL(k_slot_grow, dim3(grid_for(G, 256)), dim3(256), 0,
                     c->stream, G, n_dev, (const uint32_t*)c->sel.p,
                     (const uint8_t*)c->sel_ok.p, (const uint32_t*)c->sel_e.p,
                     (const uint32_t*)c->sel_s.p,
                     (const uint32_t*)c->cnt_tl.p, c->ne2.p, c->ns2.p,
                     c->lane_cap.p);
  int rc = hip_check(c, hipGetLastError(), "slot size launch");
  if (!rc) rc = reserve(c, c->epj_off2, (size_t)G + 1);
  if (!rc) rc = reserve(c, c->spj_off2, (size_t)G + 1);
  if (!rc) rc = reserve(c, c->lane_off2, (size_t)nl + 1);
  if (!rc) rc = scan_u32_to_u64(c, c->ne2.p, c->epj_off2.p, G);
  if (!rc) rc = scan_u32_to_u64(c, c->ns2.p, c->spj_off2.p, G);
  if (!rc) rc = scan_u32_to_u64(c, c->lane_cap.p, c->lane_off2.p, nl);
  if (!rc) rc = stage_d2h(c, 0, c->epj_off2.p + G, 8);
  if (!rc) rc = stage_d2h(c, 8, c->spj_off2.p + G, 8);
  if (!rc) rc = stage_d2h(c, 16, c->lane_off2.p + nl, 8);
  if (!rc) rc = sync_stream(c);
  if (rc) return rc;
  const uint64_t* h = static_cast<const uint64_t*>(c->h_small);
  const int64_t ce = (int64_t)h[0], cs = (int64_t)h[1];
  const int64_t lt = (int64_t)h[2];
  drop_graph(c);
  if ((rc = reserve(c, c->epj2, (size_t)ce + 1))) return rc;
  if ((rc = reserve(c, c->spj2, (size_t)cs + 1))) return rc;
  hipLaunchKernelGGL(k_slot_move, dim3(grid_for(G, 4)), dim3(256), 0,
                     c->stream, G, (const uint32_t*)c->cnt_e.p,
                     (const uint32_t*)c->cnt_s.p, (const uint64_t*)c->epj_off.p,
                     (const uint32_t*)c->epj.p, (const uint64_t*)c->spj_off.p,
                     (const uint32_t*)c->spj.p, (const uint64_t*)c->epj_off2.p,
                     c->epj2.p, (const uint64_t*)c->spj_off2.p, c->spj2.p);
  if ((rc = hip_check(c, hipGetLastError(), "slot move launch"))) return rc;
  std::swap(c->epj, c->epj2);
  std::swap(c->spj, c->spj2);
  std::swap(c->epj_off, c->epj_off2);
  std::swap(c->spj_off, c->spj_off2);
  std::swap(c->lane_off, c->lane_off2);
  c->cap_e = ce;
  c->cap_s = cs;
  c->lane_total = lt;
  return reserve(c, c->tok, (size_t)lt + 1);
}

// Selection from host ids (ascending, unique, in range: checked here).
int refresh_host_sel(nb_ctx* c, int64_t n_sel, const int64_t* sel) {
  const int64_t G = c->n_groups;
  if (n_sel < 0 || n_sel > G || (n_sel > 0 && !sel))
    return set_err(c, NB_ERR_INPUT, "bad selection size %lld", (long long)n_sel);
  std::vector<uint32_t> h((size_t)n_sel);
  for (int64_t i = 0; i < n_sel; ++i) {
    if (sel[i] < 0 || sel[i] >= G || (i > 0 && sel[i] <= sel[i - 1]))
      return set_err(c, NB_ERR_INPUT,
                     "selection must hold ascending group ids in [0, %lld)",
                     (long long)G);
    h[(size_t)i] = (uint32_t)sel[i];
  }
  int rc = launch_group_box(c, c->g_clo.p, c->g_chi.p);
  if (!rc) rc = fill_u32(c, c->pick.p, G, 0u);
  if (rc) return rc;
  if (n_sel > 0) {
    rc = hip_check(c, hipMemcpyAsync(c->sel.p, h.data(), (size_t)n_sel * 4,
                                     hipMemcpyHostToDevice, c->stream),
                   "selection upload");
    if (rc) return rc;
    hipLaunchKernelGGL(k_mark, dim3(grid_for(n_sel, 256)), dim3(256), 0,
                       c->stream, n_sel, (const uint32_t*)c->sel.p, c->pick.p);
    rc = hip_check(c, hipGetLastError(), "mark launch");
  }
  if (!rc) rc = scan_u32(c, c->pick.p, c->pickpos.p, G);
  if (rc) return rc;
  // a list that does not fit its slot is walked again into a larger one
  // (the selection's other groups get the same list again)
  for (int attempt = 0; attempt < 2; ++attempt) {
    rc = refresh_selected(c);
    if (!rc) rc = stage_d2h(c, 0, c->red.p + kRedRefreshed, 16);
    if (!rc) rc = sync_stream(c);  // also: the host vector goes out of scope
    if (rc) return rc;
    const uint64_t* done = static_cast<const uint64_t*>(c->h_small);
    const uint64_t fitted = done[0], missed = done[1];
    if (!missed) {
      c->host_refreshed += n_sel;
      return NB_OK;
    }
    if (attempt == 0 && (rc = grow_slots(c))) return rc;
    if (attempt == 1)
      return set_err(c, NB_ERR_LIST,
                     "%llu of %llu refreshed lists did not fit their groups' "
                     "list slots (those groups keep their lists)",
                     (unsigned long long)missed,
                     (unsigned long long)(fitted + missed));
  }
  return NB_OK;
}

// Predictor-driven refresh: features, perceptron, selection p > p* or
// age >= k_max, and the refresh of the selection; no host synchronisation.
int refresh_predicted(nb_ctx* c) {
  const int64_t G = c->n_groups;
  int rc = mlp_ensure(c);
  if (!rc) rc = launch_features(c);
  if (!rc) rc = mlp_forward(c, G, c->feat.p, c->prob.p);
  if (rc) return rc;
  hipLaunchKernelGGL(k_select, dim3(grid_for(G, 256)), dim3(256), 0,
                     c->stream, G, (const float*)c->prob.p,
                     (const uint32_t*)c->g_age.p, (float)c->cfg.p_star,
                     (uint32_t)c->cfg.k_max, c->pick.p);
  rc = hip_check(c, hipGetLastError(), "select launch");
  if (!rc) rc = scan_u32(c, c->pick.p, c->pickpos.p, G);
  if (rc) return rc;
  hipLaunchKernelGGL(k_compact, dim3(grid_for(G, 256)), dim3(256), 0,
                     c->stream, G, (const uint32_t*)c->pick.p,
                     (const uint32_t*)c->pickpos.p, c->sel.p);
  rc = hip_check(c, hipGetLastError(), "compact launch");
  return rc ? rc : refresh_selected(c);
}

// Refresh driven by the exact check at tolerance cfg.tau (or the age).
int refresh_checked(nb_ctx* c) {
  const int64_t G = c->n_groups;
  int rc = launch_stale(c, c->cfg.tau);
  if (rc) return rc;
  hipLaunchKernelGGL(k_select_stale, dim3(grid_for(G, 256)), dim3(256), 0,
                     c->stream, G, (const uint8_t*)c->stale.p,
                     (const uint32_t*)c->g_age.p, (uint32_t)c->cfg.k_max,
                     c->pick.p);
  rc = hip_check(c, hipGetLastError(), "select launch");
  if (!rc) rc = scan_u32(c, c->pick.p, c->pickpos.p, G);
  if (rc) return rc;
  hipLaunchKernelGGL(k_compact, dim3(grid_for(G, 256)), dim3(256), 0,
                     c->stream, G, (const uint32_t*)c->pick.p,
                     (const uint32_t*)c->pickpos.p, c->sel.p);
  rc = hip_check(c, hipGetLastError(), "compact launch");
  return rc ? rc : refresh_selected(c);
}

int labels_to_float(nb_ctx* c, float* out) {
  hipLaunchKernelGGL(k_u8_to_f32, dim3(grid_for(c->n_groups, 256)), dim3(256),
                     0, c->stream, c->n_groups, (const uint8_t*)c->stale.p,
                     out);
  return hip_check(c, hipGetLastError(), "label launch");
}

}  // namespace nb

// ---- C ABI ------------------------------------------------------------------
using namespace nb;

namespace {

int need_refresh_state(nb_ctx* c) {
  if (!c->learn)
    return set_err(c, NB_ERR_STATE, "needs a context with NB_FLAG_REFRESH");
  if (!c->tree_valid || !c->lists_valid || !c->lists_reusable)
    return set_err(c, NB_ERR_STATE,
                   "needs lists made with MAKE_LIST_FOR_REUSE");
  if (!c->shift_fresh)
    return set_err(c, NB_ERR_STATE,
                   "positions moved since the last force computation");
  return NB_OK;
}

int copy_out(nb_ctx* c, void* dst, const void* src, size_t bytes,
             int on_device) {
  int rc = hip_check(c, hipMemcpyAsync(dst, src, bytes,
                                       on_device ? hipMemcpyDeviceToDevice
                                                 : hipMemcpyDeviceToHost,
                                       c->stream),
                     "readback");
  return rc ? rc : sync_stream(c);
}

// Inputs of the perceptron calls: device pointers are used in place, host
// arrays are copied into the context's staging buffers.
int stage_in(nb_ctx* c, DBuf<float>& buf, const float* src, size_t count,
             int on_device, const float** out) {
  if (on_device) {
    *out = src;
    return NB_OK;
  }
  int rc = reserve(c, buf, count);
  if (!rc) rc = hip_check(c, hipMemcpyAsync(buf.p, src, count * 4,
                                            hipMemcpyHostToDevice, c->stream),
                          "upload");
  if (!rc) rc = sync_stream(c);
  *out = buf.p;
  return rc;
}

}  // namespace

extern "C" {

int nb_group_features(nb_ctx* c, float* feat, int on_device) {
  if (!c) return NB_ERR_INPUT;
  int rc = need_refresh_state(c);
  if (!rc) rc = launch_features(c);
  if (!rc && feat)
    rc = copy_out(c, feat, c->feat.p, (size_t)c->n_groups * NB_MLP_NIN * 4,
                  on_device);
  return rc;
}

int nb_group_stale(nb_ctx* c, double tau, uint8_t* stale, float* label,
                   int on_device) {
  if (!c) return NB_ERR_INPUT;
  if (!(tau >= 0.0) || !std::isfinite(tau))
    return set_err(c, NB_ERR_INPUT, "tau must be finite and >= 0");
  if (c->cfg.theta <= 0.0)
    return set_err(c, NB_ERR_INPUT, "staleness needs theta > 0");
  int rc = need_refresh_state(c);
  if (!rc) rc = launch_stale(c, tau);
  if (!rc && stale)
    rc = copy_out(c, stale, c->stale.p, (size_t)c->n_groups, on_device);
  if (!rc && label) {
    if (on_device) {
      rc = labels_to_float(c, label);
      if (!rc) rc = sync_stream(c);
    } else {
      std::vector<uint8_t> h((size_t)c->n_groups);
      rc = copy_out(c, h.data(), c->stale.p, h.size(), 0);
      for (size_t g = 0; !rc && g < h.size(); ++g) label[g] = (float)h[g];
    }
  }
  return rc;
}

int nb_refresh_lists(nb_ctx* c, int64_t n_sel, const int64_t* sel) {
  if (!c) return NB_ERR_INPUT;
  int rc = need_refresh_state(c);
  if (rc) return rc;
  Timed t(c, NB_PH_REFRESH);
  return refresh_host_sel(c, n_sel, sel);
}

int nb_get_group_state(nb_ctx* c, double* sa, double* so, int32_t* age) {
  if (!c) return NB_ERR_INPUT;
  if (!c->learn || !c->lists_valid)
    return set_err(c, NB_ERR_STATE, "needs NB_FLAG_REFRESH and lists");
  const size_t ng = (size_t)c->n_groups;
  int rc = NB_OK;
  if (sa) rc = copy_out(c, sa, c->g_sa.p, ng * 8, 0);
  if (!rc && so) rc = copy_out(c, so, c->g_so.p, ng * 8, 0);
  if (!rc && age) {
    std::vector<uint32_t> h(ng);
    rc = copy_out(c, h.data(), c->g_age.p, ng * 4, 0);
    for (size_t g = 0; !rc && g < ng; ++g)
      age[g] = (int32_t)(h[g] > 0x7FFFFFFFu ? 0x7FFFFFFFu : h[g]);
  }
  return rc;
}

int nb_get_cell_sides(nb_ctx* c, double* side) {
  if (!c || !side) return NB_ERR_INPUT;
  if (!c->learn || !c->tree_valid || !c->shift_fresh)
    return set_err(c, NB_ERR_STATE,
                   "needs NB_FLAG_REFRESH and moments of the current positions");
  std::vector<double4> h((size_t)c->n_cell);
  int rc = copy_out(c, h.data(), c->c_shift.p, h.size() * sizeof(double4), 0);
  for (size_t i = 0; !rc && i < h.size(); ++i) side[i] = h[i].w;
  return rc;
}

int nb_mlp_set(nb_ctx* c, const float* w, int64_t nw) {
  if (!c || !w) return NB_ERR_INPUT;
  if (nw != NB_MLP_NPARAM)
    return set_err(c, NB_ERR_INPUT, "expected %d parameters", NB_MLP_NPARAM);
  int rc = mlp_ensure(c);
  if (!rc) rc = hip_check(c, hipMemcpyAsync(c->mlp_w.p, w, NB_MLP_NPARAM * 4,
                                            hipMemcpyHostToDevice, c->stream),
                          "weight upload");
  if (!rc) rc = hip_check(c, hipMemsetAsync(c->mlp_m.p, 0, NB_MLP_NPARAM * 4,
                                            c->stream), "adam reset");
  if (!rc) rc = hip_check(c, hipMemsetAsync(c->mlp_v.p, 0, NB_MLP_NPARAM * 4,
                                            c->stream), "adam reset");
  if (!rc) rc = sync_stream(c);
  c->mlp_t = 0;
  return rc;
}

int nb_mlp_get(nb_ctx* c, float* w, int64_t nw) {
  if (!c || !w) return NB_ERR_INPUT;
  if (nw != NB_MLP_NPARAM)
    return set_err(c, NB_ERR_INPUT, "expected %d parameters", NB_MLP_NPARAM);
  int rc = mlp_ensure(c);
  if (!rc) rc = copy_out(c, w, c->mlp_w.p, NB_MLP_NPARAM * 4, 0);
  return rc;
}

int nb_mlp_forward(nb_ctx* c, int64_t n, const float* x, float* p,
                   int on_device) {
  if (!c) return NB_ERR_INPUT;
  if (n < 0 || (n > 0 && (!x || !p)))
    return set_err(c, NB_ERR_INPUT, "bad perceptron input");
  if (n == 0) return NB_OK;
  int rc = mlp_ensure(c);
  const float* xd = nullptr;
  if (!rc) rc = stage_in(c, c->mlp_x, x, (size_t)n * NB_MLP_NIN, on_device, &xd);
  if (rc) return rc;
  float* pd = p;
  if (!on_device) {
    if ((rc = reserve(c, c->mlp_y, (size_t)n))) return rc;
    pd = c->mlp_y.p;
  }
  rc = mlp_forward(c, n, xd, pd);
  if (!rc) rc = on_device ? sync_stream(c) : copy_out(c, p, pd, (size_t)n * 4, 0);
  return rc;
}

int nb_mlp_grad(nb_ctx* c, int64_t n, const float* x, const float* y,
                float pos_weight, float* loss, float* grad, int on_device) {
  if (!c) return NB_ERR_INPUT;
  if (n < 1 || !x || !y || !(pos_weight > 0.f))
    return set_err(c, NB_ERR_INPUT, "bad perceptron input");
  int rc = mlp_ensure(c);
  const float *xd = nullptr, *yd = nullptr;
  if (!rc) rc = stage_in(c, c->mlp_x, x, (size_t)n * NB_MLP_NIN, on_device, &xd);
  if (!rc) rc = stage_in(c, c->mlp_y, y, (size_t)n, on_device, &yd);
  if (!rc) rc = mlp_grad(c, n, xd, yd, pos_weight);
  if (rc) return rc;
  if (grad) rc = copy_out(c, grad, c->mlp_g.p, NB_MLP_NPARAM * 4, on_device);
  if (!rc && loss) rc = copy_out(c, loss, c->mlp_g.p + NB_MLP_NPARAM, 4, 0);
  if (!rc) rc = sync_stream(c);
  return rc;
}

int nb_mlp_grad_static(nb_ctx* c, int64_t n, const float* x, const float* y,
                       float pos_weight, float* loss, float* grad) {
  if (!c) return NB_ERR_INPUT;
  if (n < 1 || n > NB_MLP_STATIC_MAX_ROWS || !x || !y || !grad ||
      !(pos_weight > 0.f))
    return set_err(c, NB_ERR_INPUT,
                   "bad perceptron input (1 <= n <= %d device rows, x, y and "
                   "grad required, pos_weight > 0)", NB_MLP_STATIC_MAX_ROWS);
  if (!c->mlp_w.p)
    return set_err(c, NB_ERR_STATE, "no perceptron weights (nb_mlp_set first)");
  float* s = (c->device >= 0 && c->device < kMaxDevices)
                 ? g_scratch_dev[c->device] : nullptr;
  if (!s) return set_err(c, NB_ERR_STATE, "static scratch not set up");
  return mlp_grad_into(c, n, x, y, pos_weight, s + kSAct, s + kSDz,
                       s + kSLoss, s + kSPart, grad, loss ? loss : s + kSSink);
}

int nb_mlp_adam(nb_ctx* c, const float* grad, float lr, float beta1,
                float beta2, float eps, int on_device) {
  if (!c) return NB_ERR_INPUT;
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return set_err(c, NB_ERR_INPUT, "bad Adam parameters");
  int rc = mlp_ensure(c);
  const float* gd = c->mlp_g.p;
  if (!rc && grad) rc = stage_in(c, c->mlp_part, grad, NB_MLP_NPARAM, on_device, &gd);
  if (!rc) rc = mlp_adam(c, gd, lr, beta1, beta2, eps);
  if (!rc) rc = sync_stream(c);
  return rc;
}

int nb_mlp_train(nb_ctx* c, int64_t n, const float* x, const float* y,
                 int on_device, int epochs, int64_t batch, float lr,
                 float pos_weight, float* loss) {
  if (!c) return NB_ERR_INPUT;
  if (n < 1 || !x || !y || epochs < 1 || batch < 1 || !(lr > 0.f) ||
      !(pos_weight > 0.f))
    return set_err(c, NB_ERR_INPUT, "bad training input");
  int rc = mlp_ensure(c);
  const float *xd = nullptr, *yd = nullptr;
  // host data: both arrays go to the two staging buffers; the gradient
  // scratch is separate
  if (!rc) rc = stage_in(c, c->mlp_x, x, (size_t)n * NB_MLP_NIN, on_device, &xd);
  if (!rc) rc = stage_in(c, c->mlp_y, y, (size_t)n, on_device, &yd);
  for (int e = 0; !rc && e < epochs; ++e) {
    for (int64_t b0 = 0; !rc && b0 < n; b0 += batch) {
      const int64_t nb = b0 + batch < n ? batch : n - b0;
      rc = mlp_grad(c, nb, xd + (size_t)b0 * NB_MLP_NIN, yd + b0, pos_weight);
      if (!rc) rc = mlp_adam(c, c->mlp_g.p, lr, 0.9f, 0.999f, 1e-8f);
    }
  }
  if (!rc && loss) {
    rc = mlp_grad(c, n, xd, yd, pos_weight);
    if (!rc) rc = copy_out(c, loss, c->mlp_g.p + NB_MLP_NPARAM, 4, 0);
  }
  if (!rc) rc = sync_stream(c);
  return rc;
}

}  // extern "C"
