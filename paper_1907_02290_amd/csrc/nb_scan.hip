// nb_scan.hip -- device-wide exclusive scans and the stable LSD radix sort
// of (Morton key, index) pairs (section 4.3, local tree step 2: radix sort
// with 8-bit digits, eight passes over 64-bit keys).
//
// Radix pass = upsweep (per-block digit histograms) + per-digit scan over
// blocks + downsweep.  The downsweep ranks keys stably inside a block with
// wave64 ballots (the lanes that share a digit are found bit by bit), stages
// the block's keys in LDS in digit order and writes them out so that equal
// digits land in contiguous, coalesced runs.
#include <utility>

#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__device__ inline T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive scan across the block (blockDim.x multiple of 64, <= 1024).
template <class T>
__device__ inline T block_excl_scan(T v, T* lds, T* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  T inc = wave_incl_scan(v);
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  T wbase = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    T s = lds[i];
    if (i < w) wbase += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return wbase + inc - v;
}

template <class Tin, class Tacc>
__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(const Tin* __restrict__ in, int64_t n, Tacc* __restrict__ bs) {
  __shared__ Tacc lds[16];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  Tacc s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
    if (i < n) s += (Tacc)in[i];
  }
  Tacc tot;
  block_excl_scan<Tacc>(s, lds, &tot);
  if (threadIdx.x == 0) bs[blockIdx.x] = tot;
}

template <class Tacc>
__global__ void __launch_bounds__(1024) k_scan_top(Tacc* bs, int64_t nb) {
  __shared__ Tacc lds[16];
  const int64_t per = (nb + blockDim.x - 1) / blockDim.x;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  Tacc s = 0;
  for (int64_t i = b0; i < b0 + per && i < nb; ++i) s += bs[i];
  Tacc tot;
  Tacc run = block_excl_scan<Tacc>(s, lds, &tot);
  for (int64_t i = b0; i < b0 + per && i < nb; ++i) {
    Tacc v = bs[i];
    bs[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) bs[nb] = tot;
}

// out[i] = sum of in[0..i); out[n] = total.  in == out is allowed.
template <class Tin, class Tout, class Tacc>
__global__ void __launch_bounds__(kScanThreads)
k_scan_down(const Tin* in, Tout* out, int64_t n, const Tacc* __restrict__ bs,
            int64_t nb) {
  __shared__ Tacc lds[16];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int64_t my = base + (int64_t)threadIdx.x * kScanItems;
  Tacc v[kScanItems];
  Tacc s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (my + j < n) ? (Tacc)in[my + j] : (Tacc)0;
    s += v[j];
  }
  Tacc tot;
  Tacc run = block_excl_scan<Tacc>(s, lds, &tot) + bs[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (my + j < n) out[my + j] = (Tout)run;
    run += v[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (Tout)bs[nb];
}

template <class Tin, class Tout, class Tacc>
int scan_impl(nb_ctx* c, const Tin* in, Tout* out, int64_t n) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  int rc = reserve(c, c->scan_tmp, (size_t)nb + 1);
  if (rc) return rc;
  Tacc* bs = reinterpret_cast<Tacc*>(c->scan_tmp.p);
  static_assert(sizeof(Tacc) <= sizeof(uint64_t), "scan accumulator");
  if (nb > 0) {
    hipLaunchKernelGGL((k_scan_reduce<Tin, Tacc>), dim3((unsigned)nb),
                       dim3(kScanThreads), 0, c->stream, in, n, bs);
  }
  hipLaunchKernelGGL((k_scan_top<Tacc>), dim3(1), dim3(1024), 0, c->stream,
                     bs, nb);
  hipLaunchKernelGGL((k_scan_down<Tin, Tout, Tacc>),
                     dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kScanThreads), 0,
                     c->stream, in, out, n, (const Tacc*)bs, nb);
  return hip_check(c, hipGetLastError(), "scan launch");
}

// ---------------------------------------------------------------------------
// Radix sort
constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsRows = 16;                      // rows of 64 keys per wave
constexpr int kRsTile = kRsThreads * kRsRows;    // 4096 keys per block

// Digit of an element: 8 bits of its Morton key, or (SYS) 8 bits of the
// system id of the slot it came from -- the last passes group the systems
// while keeping each system's Morton order.
template <bool SYS>
__device__ inline uint32_t rs_digit(uint64_t k, uint32_t v,
                                    const uint32_t* __restrict__ seg,
                                    int shift) {
  return SYS ? (seg[v] >> shift) & 255u : (uint32_t)(k >> shift) & 255u;
}

template <bool SYS>
__global__ void __launch_bounds__(kRsThreads)
k_rs_upsweep(const uint64_t* __restrict__ key,
             const uint32_t* __restrict__ val,
             const uint32_t* __restrict__ seg, int64_t n, int shift,
             uint32_t* __restrict__ hist, int nblk) {
  __shared__ uint32_t h[kRsWaves][256];
  const int t = threadIdx.x, w = t >> 6;
  for (int i = t; i < kRsWaves * 256; i += kRsThreads) (&h[0][0])[i] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
  for (int j = 0; j < kRsRows; ++j) {
    const int64_t idx = base + (int64_t)j * kRsThreads + t;
    if (idx < n) {
      const uint32_t d =
          rs_digit<SYS>(SYS ? 0ull : key[idx],
                        SYS ? (val ? val[idx] : (uint32_t)idx) : 0u, seg,
                        shift);
      atomicAdd(&h[w][d], 1u);
    }
  }
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kRsWaves; ++i) s += h[i][t];
  hist[(int64_t)t * nblk + blockIdx.x] = s;
}

// One block per digit: exclusive scan of that digit's block counts.
__global__ void __launch_bounds__(256)
k_rs_scan_digit(uint32_t* __restrict__ hist, int nblk,
                uint32_t* __restrict__ dtot) {
  __shared__ uint32_t lds[16];
  uint32_t* row = hist + (int64_t)blockIdx.x * nblk;
  const int per = (nblk + 255) / 256;
  const int b0 = threadIdx.x * per;
  uint32_t s = 0;
  for (int i = b0; i < b0 + per && i < nblk; ++i) s += row[i];
  uint32_t tot;
  uint32_t run = block_excl_scan<uint32_t>(s, lds, &tot);
  for (int i = b0; i < b0 + per && i < nblk; ++i) {
    uint32_t v = row[i];
    row[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = tot;
}

template <bool SYS>
__global__ void __launch_bounds__(kRsThreads)
k_rs_downsweep(const uint64_t* __restrict__ key_in,
               const uint32_t* __restrict__ val_in,
               const uint32_t* __restrict__ seg,
               uint64_t* __restrict__ key_out, uint32_t* __restrict__ val_out,
               int64_t n, int shift, const uint32_t* __restrict__ hist,
               const uint32_t* __restrict__ dtot, int nblk) {
  __shared__ uint64_t s_key[kRsTile];
  __shared__ uint32_t s_val[kRsTile];
  __shared__ uint32_t whist[kRsWaves][256];
  __shared__ uint32_t lbase[kRsWaves][256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t lds[16];

  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int i = t; i < kRsWaves * 256; i += kRsThreads) (&whist[0][0])[i] = 0;
  __syncthreads();

  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t k[kRsRows];
  uint32_t v[kRsRows];
  uint32_t loc[kRsRows];
#pragma unroll
  for (int j = 0; j < kRsRows; ++j) {
    const int64_t idx = base + (int64_t)(w * kRsRows + j) * 64 + lane;
    const bool ok = idx < n;
    k[j] = ok ? key_in[idx] : 0ull;
    v[j] = ok ? (val_in ? val_in[idx] : (uint32_t)idx) : 0u;
  }
#pragma unroll
  for (int j = 0; j < kRsRows; ++j) {
    const int64_t idx = base + (int64_t)(w * kRsRows + j) * 64 + lane;
    const bool ok = idx < n;
    const uint32_t d = ok ? rs_digit<SYS>(k[j], v[j], seg, shift) : 0u;
    uint64_t peer = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peer &= bit ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peer & lt_mask);
    const uint32_t cnt = (uint32_t)__popcll(peer);
    uint32_t wb = 0;
    if (ok) wb = whist[w][d];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (ok && rank == 0) whist[w][d] = wb + cnt;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    loc[j] = wb + rank;
  }
  __syncthreads();
  {
    const int d = t;  // 256 threads, one digit each
    uint32_t cw[kRsWaves];
    uint32_t tot = 0;
#pragma unroll
    for (int i = 0; i < kRsWaves; ++i) {
      cw[i] = whist[i][d];
      tot += cw[i];
    }
    uint32_t all;
    const uint32_t start = block_excl_scan<uint32_t>(tot, lds, &all);
    uint32_t r = start;
#pragma unroll
    for (int i = 0; i < kRsWaves; ++i) {
      lbase[i][d] = r;
      r += cw[i];
    }
    uint32_t all2;
    const uint32_t dbase = block_excl_scan<uint32_t>(dtot[d], lds, &all2);
    gbase[d] = dbase + hist[(int64_t)d * nblk + blockIdx.x] - start;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kRsRows; ++j) {
    const int64_t idx = base + (int64_t)(w * kRsRows + j) * 64 + lane;
    if (idx < n) {
      const uint32_t d = rs_digit<SYS>(k[j], v[j], seg, shift);
      const uint32_t p = lbase[w][d] + loc[j];
      s_key[p] = k[j];
      s_val[p] = v[j];
    }
  }
  __syncthreads();
  const int64_t rem = n - base;
  const int tile_n = (int)(rem < kRsTile ? rem : kRsTile);
  for (int i = t; i < tile_n; i += kRsThreads) {
    const uint64_t kk = s_key[i];
    const uint32_t d = rs_digit<SYS>(kk, s_val[i], seg, shift);
    const uint32_t dest = gbase[d] + (uint32_t)i;
    key_out[dest] = kk;
    val_out[dest] = s_val[i];
  }
}

}  // namespace

int scan_u32(nb_ctx* c, const uint32_t* in, uint32_t* out, int64_t n) {
  return scan_impl<uint32_t, uint32_t, uint32_t>(c, in, out, n);
}

int scan_u32_to_u64(nb_ctx* c, const uint32_t* in, uint64_t* out, int64_t n) {
  return scan_impl<uint32_t, uint64_t, uint64_t>(c, in, out, n);
}

// Sorts c->key / c->val (first n entries) ascending by key, stably; the
// initial values are the slot indices 0..n-1.  Eight 8-bit passes cover the
// 63-bit keys.  With several systems, one more stable pass per 8 bits of the
// system id groups the systems (each keeps its slots [off_s, off_s+1)).  The
// result is left in c->key / c->val.
int radix_sort(nb_ctx* c, int64_t n) {
  const int nblk = (int)((n + kRsTile - 1) / kRsTile);
  int rc = reserve(c, c->hist, (size_t)256 * nblk);
  if (!rc) rc = reserve(c, c->dtot, 256);
  if (!rc) rc = reserve(c, c->key2, (size_t)n);
  if (!rc) rc = reserve(c, c->val2, (size_t)n);
  if (rc) return rc;
  int sys_passes = 0;
  for (int64_t m = c->n_sys - 1; m > 0; m >>= 8) ++sys_passes;
  uint64_t* kin = c->key.p;
  uint64_t* kout = c->key2.p;
  uint32_t* vin = nullptr;  // first pass: implicit iota
  uint32_t* vout = c->val2.p;
  const uint32_t* seg = c->seg.p;
  for (int pass = 0; pass < 8 + sys_passes; ++pass) {
    const bool sys = pass >= 8;
    const int shift = sys ? 8 * (pass - 8) : 8 * pass;
    if (sys) {
      hipLaunchKernelGGL(k_rs_upsweep<true>, dim3(nblk), dim3(kRsThreads), 0,
                         c->stream, (const uint64_t*)kin, (const uint32_t*)vin,
                         seg, n, shift, c->hist.p, nblk);
    } else {
      hipLaunchKernelGGL(k_rs_upsweep<false>, dim3(nblk), dim3(kRsThreads), 0,
                         c->stream, (const uint64_t*)kin, (const uint32_t*)vin,
                         seg, n, shift, c->hist.p, nblk);
    }
    hipLaunchKernelGGL(k_rs_scan_digit, dim3(256), dim3(256), 0, c->stream,
                       c->hist.p, nblk, c->dtot.p);
    if (sys) {
      hipLaunchKernelGGL(k_rs_downsweep<true>, dim3(nblk), dim3(kRsThreads),
                         0, c->stream, (const uint64_t*)kin,
                         (const uint32_t*)vin, seg, kout, vout, n, shift,
                         (const uint32_t*)c->hist.p,
                         (const uint32_t*)c->dtot.p, nblk);
    } else {
      hipLaunchKernelGGL(k_rs_downsweep<false>, dim3(nblk), dim3(kRsThreads),
                         0, c->stream, (const uint64_t*)kin,
                         (const uint32_t*)vin, seg, kout, vout, n, shift,
                         (const uint32_t*)c->hist.p,
                         (const uint32_t*)c->dtot.p, nblk);
    }
    std::swap(kin, kout);
    if (pass == 0) {
      vin = vout;
      vout = c->val.p;
    } else {
      std::swap(vin, vout);
    }
  }
  // the sorted data is in (kin, vin); make it c->key / c->val
  if (kin != c->key.p) std::swap(c->key, c->key2);
  if (vin != c->val.p) std::swap(c->val, c->val2);
  if (kin != c->key.p || vin != c->val.p)
    return set_err(c, NB_ERR_HIP, "radix sort buffer parity");
  return hip_check(c, hipGetLastError(), "radix sort launch");
}

}  // namespace nb
