// Batched fast Gauss transforms on gfx950: B independent transforms of uneven
// sizes, each with its own delta, and R strength columns, in one fixed launch
// sequence (no host synchronisation, no allocation: it can be captured in a
// HIP graph and replayed).
//
// Transform b has targets x[x_off_b ..), sources y[y_off_b ..), strengths
// alpha[(y_off_b + j) * R + r] and outputs u[(x_off_b + i) * R + r].  Its
// coordinates are scaled by s_b = 1/sqrt(delta_b), which turns its kernel into
// exp(-z^2/4) and lets every transform use the one SOE table at delta = 1
// (the nodes of (1.3) scale exactly as 1/sqrt(delta)).
//
// Sort (each transform on its own; Section 4's sort of sources and targets):
//   k_seg_minmax    per transform: range [lo, hi] of the scaled coordinates
//   k_seg_count     per chunk of kBChunk merged points: counts per bucket,
//                   a bucket being the top bits of the key
//                   q = (z' - lo) 2^62 / (hi - lo)
//   k_seg_offsets   per transform: exclusive offsets, bucket-major, so the
//                   split is stable
//   k_seg_scatter   per chunk: stable ranks inside the chunk, merged indices
//                   and coordinates written side by side to their bucket
//   k_bucket_sort   per bucket: LSD radix sort of its keys in LDS, each with
//                   its position in the bucket (a bucket above kBucketMax
//                   points, possible only for very uneven data, is sorted by
//                   the same block through global memory), then the sorted
//                   coordinates and the output codes read from the bucket.
// The gaps are scaled only in the scan, (z_p - z_{p-1}) / sqrt(delta_b), so
// that their rounding error is relative to the gap, as in the single path.
// Key digits below the allowed sort resolution are not sorted (the same
// criterion as the single-transform path).
//
// Scan: the sorted points of all transforms form one sequence; the factor
// e_p = exp(-tau (z_p - z_{p-1})) is set to 0 at the first point of each
// transform, which decouples the transforms exactly: h+ restarts there and
// h- stops there.  So the reduce-then-scan of the single path applies to the
// whole batch at once, with one exponential per (point, mode) shared by all R
// columns:
//   k_bscan<REDUCE>  per tile: the tile's map (A, F_r, G_r) for every mode and column
//   carries          the three-level tile carries over modes x columns scans
//   k_bscan<FINAL>   per tile: chunk maps, scans across chunks, sweeps, sum over
//                    modes, u rows written for the targets.
#include <string.h>

#include "fgt_device.h"

namespace fgt {
namespace {

constexpr uint32_t kPad = 0xffffffffu;   // code of a position past the last point

__device__ __forceinline__ double seg_point(const SegInfo& sg, const double* __restrict__ x,
                                            const double* __restrict__ y, int64_t p) {
  return p < sg.N ? y[sg.y_off + p] : x[sg.x_off + (p - sg.N)];
}

__device__ __forceinline__ double qscale(double lo, double hi) {
  const double qs = hi > lo ? 4.611686018427387904e18 / (hi - lo) : 0.0;   // 2^62 / range
  return isfinite(qs) ? qs : 0.0;
}

// Key of a coordinate.  Counting and scattering must see bit-identical keys,
// so the operations are never contracted into fused multiply-adds (whose
// rounding could then differ between the kernels it is inlined into).
__device__ __forceinline__ uint64_t quant_key(double z, double scale, double lo, double qs) {
#pragma clang fp contract(off)
  const double zp = z * scale;
  double v = (zp - lo) * qs;
  v = v > 0.0 ? v : 0.0;
  v = v < 4.611686018427387904e18 ? v : 4.611686018427387904e18;
  return (uint64_t)v;
}

__device__ __forceinline__ uint64_t point_key(const SegInfo& sg, const double* __restrict__ x,
                                              const double* __restrict__ y, int64_t p, double lo,
                                              double qs) {
  return quant_key(seg_point(sg, x, y, p), sg.scale, lo, qs);
}

__device__ __forceinline__ uint32_t bucket_of(uint64_t q, int nb_log2) {
  if (nb_log2 == 0) return 0u;
  const uint32_t b = (uint32_t)(q >> (62 - nb_log2));
  const uint32_t top = (1u << nb_log2) - 1u;
  return b < top ? b : top;
}

// Lowest key bit that needs sorting: keys differing only below it belong to
// points closer than s_allow (scaled units), which may stay unordered.
__device__ __forceinline__ int resolution_bits(double lo, double hi, double s_allow) {
  const double qs = qscale(lo, hi);
  if (qs == 0.0) return 64;                 // all keys equal
  const double units = s_allow * qs;        // key units within s_allow
  if (!(units >= 1.0)) return 0;
  const int b = (int)floor(log2(units));
  return b < 62 ? b : 62;
}

// ---------------------------------------------------------------------------
// Sort kernels.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_seg_minmax(const SegInfo* __restrict__ seg,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    double* __restrict__ lo,
                                                    double* __restrict__ hi,
                                                    uint32_t* __restrict__ status) {
  __shared__ double smin[4], smax[4];
  const SegInfo sg = seg[blockIdx.x];
  const int64_t P = sg.M + sg.N;
  double mn = INFINITY, mx = -INFINITY;
  bool bad = false;
  constexpr int kBatch = 8;   // loads issued together before they are used
  for (int64_t p0 = threadIdx.x; p0 < P; p0 += 256 * kBatch) {
    double zb[kBatch];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int64_t p = p0 + i * 256;
      zb[i] = p < P ? seg_point(sg, x, y, p) : seg_point(sg, x, y, p0);
    }
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const double z = zb[i] * sg.scale;
      bad |= !isfinite(z);
      mn = fmin(mn, z);
      mx = fmax(mx, z);
    }
  }
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, kWave));
    mx = fmax(mx, __shfl_xor(mx, o, kWave));
  }
  if (threadIdx.x % kWave == 0) {
    smin[threadIdx.x / kWave] = mn;
    smax[threadIdx.x / kWave] = mx;
  }
  if (bad) atomicOr(status, kStatusNonFinite);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      mn = fmin(smin[0], smin[w]);
      smin[0] = mn;
      mx = fmax(smax[0], smax[w]);
      smax[0] = mx;
    }
    lo[blockIdx.x] = smin[0];
    hi[blockIdx.x] = smax[0];
  }
}

__global__ __launch_bounds__(256) void k_seg_count(const SegInfo* __restrict__ seg,
                                                   const ChunkInfo* __restrict__ chunks,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ lo,
                                                   const double* __restrict__ hi,
                                                   uint32_t* __restrict__ counts) {
  extern __shared__ uint32_t hist[];
  const ChunkInfo ch = chunks[blockIdx.x];
  const SegInfo sg = seg[ch.seg];
  const int nb = 1 << sg.nb_log2;
  for (int i = threadIdx.x; i < nb; i += 256) hist[i] = 0u;
  __syncthreads();
  const double l = lo[ch.seg];
  const double qs = qscale(l, hi[ch.seg]);
  const int64_t P = sg.M + sg.N;
  const int64_t end = ch.start + kBChunk < P ? ch.start + kBChunk : P;
  // All of the thread's loads first, then the keys.
  constexpr int kPer = kBChunk / 256;
  double z[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int64_t p = ch.start + threadIdx.x + r * 256;
    z[r] = p < end ? seg_point(sg, x, y, p) : 0.0;
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r)
    if (ch.start + threadIdx.x + r * 256 < end)
      atomicAdd(&hist[bucket_of(quant_key(z[r], sg.scale, l, qs), sg.nb_log2)], 1u);
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x - sg.chunk0;
  for (int i = threadIdx.x; i < nb; i += 256)
    counts[sg.cnt0 + (int64_t)i * sg.n_chunks + c] = hist[i];
}

// Exclusive offsets of each (bucket, chunk) inside the transform, bucket-major.
__global__ __launch_bounds__(256) void k_seg_offsets(const SegInfo* __restrict__ seg,
                                                     const uint32_t* __restrict__ counts,
                                                     uint32_t* __restrict__ offs,
                                                     uint32_t* __restrict__ bstart,
                                                     uint32_t* __restrict__ bsize) {
  __shared__ uint32_t wsum[4];
  const SegInfo sg = seg[blockIdx.x];
  const int nb = 1 << sg.nb_log2;
  const int64_t nc = sg.n_chunks;
  const int64_t len = (int64_t)nb * nc;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  if (nc == 0) {
    for (int i = tid; i < nb; i += 256) {
      bstart[sg.bucket0 + i] = 0u;
      bsize[sg.bucket0 + i] = 0u;
    }
    return;
  }
  const int64_t per = (len + 255) / 256;
  const int64_t a0 = (int64_t)tid * per;
  const int64_t a1 = a0 + per < len ? a0 + per : len;
  uint32_t mine = 0u;
  for (int64_t i = a0; i < a1; ++i) mine += counts[sg.cnt0 + i];
  uint32_t inc = mine;
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t v = __shfl_up(inc, (unsigned)o, kWave);
    if (lane >= o) inc += v;
  }
  if (lane == kWave - 1) wsum[wave] = inc;
  __syncthreads();
  uint32_t run = inc - mine;
  for (int w = 0; w < wave; ++w) run += wsum[w];
  for (int64_t i = a0; i < a1; ++i) {
    const uint32_t c = counts[sg.cnt0 + i];
    offs[sg.cnt0 + i] = run;
    run += c;
  }
  __syncthreads();
  const uint32_t P = (uint32_t)(sg.M + sg.N);
  for (int i = tid; i < nb; i += 256) {
    const uint32_t s0 = offs[sg.cnt0 + (int64_t)i * nc];
    const uint32_t s1 = i + 1 < nb ? offs[sg.cnt0 + (int64_t)(i + 1) * nc] : P;
    bstart[sg.bucket0 + i] = s0;
    bsize[sg.bucket0 + i] = s1 - s0;
  }
}

// Stable split of one chunk into the buckets of its transform.  Wave w owns
// the chunk's items [w * kBChunk/4, (w+1) * kBChunk/4) in rounds of 64.
__global__ __launch_bounds__(256) void k_seg_scatter(const SegInfo* __restrict__ seg,
                                                     const ChunkInfo* __restrict__ chunks,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ lo,
                                                     const double* __restrict__ hi,
                                                     const uint32_t* __restrict__ offs,
                                                     uint32_t* __restrict__ ids_tmp,
                                                     double* __restrict__ z_tmp) {
  extern __shared__ uint32_t wcnt[];   // [4][nb]
  constexpr int kRounds = kBChunk / 4 / kWave;   // 16
  const ChunkInfo ch = chunks[blockIdx.x];
  const SegInfo sg = seg[ch.seg];
  const int nb = 1 << sg.nb_log2;
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  for (int i = tid; i < 4 * nb; i += 256) wcnt[i] = 0u;
  __syncthreads();
  const double l = lo[ch.seg];
  const double qs = qscale(l, hi[ch.seg]);
  const int64_t P = sg.M + sg.N;
  const int64_t end = ch.start + kBChunk < P ? ch.start + kBChunk : P;
  uint32_t bk[kRounds], rank[kRounds];
  double z[kRounds];   // all loads first
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t p = ch.start + (int64_t)wave * (kBChunk / 4) + r * kWave + lane;
    z[r] = p < end ? seg_point(sg, x, y, p) : 0.0;
  }
  for (int r = 0; r < kRounds; ++r) {
    const int64_t p = ch.start + (int64_t)wave * (kBChunk / 4) + r * kWave + lane;
    const bool valid = p < end;
    const uint32_t b = valid ? bucket_of(quant_key(z[r], sg.scale, l, qs), sg.nb_log2) : 0u;
    const uint64_t live = __ballot(valid);
    uint32_t pl = (uint32_t)live, ph = (uint32_t)(live >> 32);
    for (int bit = 0; bit < sg.nb_log2; ++bit) {   // lanes with the same bucket, as in block_rank
      const int32_t m = (int32_t)(b << (31 - bit)) >> 31;
      const uint64_t bal = __ballot(m < 0);
      pl &= ~((uint32_t)bal ^ (uint32_t)m);
      ph &= ~((uint32_t)(bal >> 32) ^ (uint32_t)m);
    }
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(ph, __builtin_amdgcn_mbcnt_lo(pl, 0u));
    const uint32_t cnt = (uint32_t)__popc(pl) + (uint32_t)__popc(ph);
    const uint32_t before = valid ? wcnt[wave * nb + b] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0u) wcnt[wave * nb + b] = before + cnt;
    __builtin_amdgcn_wave_barrier();
    bk[r] = b;
    rank[r] = valid ? before + below : kPad;
  }
  __syncthreads();
  for (int i = tid; i < nb; i += 256) {
    uint32_t run = 0u;
    for (int w = 0; w < 4; ++w) {
      const uint32_t c = wcnt[w * nb + i];
      wcnt[w * nb + i] = run;
      run += c;
    }
  }
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x - sg.chunk0;
  for (int r = 0; r < kRounds; ++r) {
    if (rank[r] == kPad) continue;
    const int64_t p = ch.start + (int64_t)wave * (kBChunk / 4) + r * kWave + lane;
    const uint64_t pos = (uint64_t)offs[sg.cnt0 + (int64_t)bk[r] * sg.n_chunks + c] +
                         wcnt[wave * nb + bk[r]] + rank[r];
    if (pos < (uint64_t)P) {
      ids_tmp[sg.base + (int64_t)pos] = (uint32_t)p;
      z_tmp[sg.base + (int64_t)pos] = z[r];
    }
  }
}

// LDS state of the block ranking below.
struct RankLds {
  uint32_t wcnt[kBSortThreads / kWave][kRadix];
  uint32_t thist[kRadix];
  uint32_t tstart[kRadix];
  uint32_t wsum[kRadix / kWave];
};

// Stable ranking of up to kBucketMax keys held kBSortItems per thread, items
// ordered (wave, item, lane), by the 8-bit digit at `shift`.  On return
// pos[i] is the item's position in digit order (for valid items), and
// lds.thist / lds.tstart hold the digit counts and exclusive starts.  A wave
// with no valid item passes wave_active = false and only joins the barriers.
__device__ __forceinline__ void block_rank(const uint64_t* key, const bool* valid, int shift,
                                           bool wave_active, uint32_t* pos, RankLds& lds) {
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  constexpr int W = kBSortThreads / kWave;
  for (int i = tid; i < W * kRadix; i += kBSortThreads) (&lds.wcnt[0][0])[i] = 0u;
  __syncthreads();
  uint32_t rank[kBSortItems];
#pragma unroll
  for (int i = 0; i < kBSortItems; ++i) rank[i] = 0u;
  // A wave whose items all lie past the end ranks nothing (uniform branch).
  if (wave_active) {
#pragma unroll
  for (int i = 0; i < kBSortItems; ++i) {
    const uint32_t dig = (uint32_t)(key[i] >> shift) & 0xffu;
    // Lanes with the same digit: per digit bit, the ballot where the lane's
    // bit is set, else its complement (ballot XOR the bit as a sign mask).
    const uint64_t live = __ballot(valid[i]);
    uint32_t pl = (uint32_t)live, ph = (uint32_t)(live >> 32);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const int32_t m = (int32_t)(dig << (31 - bit)) >> 31;
      const uint64_t bal = __ballot(m < 0);
      pl &= ~((uint32_t)bal ^ (uint32_t)m);
      ph &= ~((uint32_t)(bal >> 32) ^ (uint32_t)m);
    }
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(ph, __builtin_amdgcn_mbcnt_lo(pl, 0u));
    const uint32_t cnt = (uint32_t)__popc(pl) + (uint32_t)__popc(ph);
    const uint32_t before = lds.wcnt[wave][dig];
    __builtin_amdgcn_wave_barrier();
    if (valid[i] && below == 0u) lds.wcnt[wave][dig] = before + cnt;
    __builtin_amdgcn_wave_barrier();
    rank[i] = before + below;
  }
  }
  __syncthreads();
  if (tid < kRadix) {
    // The tile's count of digit tid is the sum of the waves' counts; they
    // become exclusive wave offsets.
    uint32_t c = 0u;
    for (int w = 0; w < W; ++w) {
      const uint32_t v = lds.wcnt[w][tid];
      lds.wcnt[w][tid] = c;
      c += v;
    }
    lds.thist[tid] = c;
    uint32_t inc = c;
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t v = __shfl_up(inc, (unsigned)o, kWave);
      if (lane >= o) inc += v;
    }
    if (lane == kWave - 1) lds.wsum[wave] = inc;
    lds.tstart[tid] = inc - c;   // completed below with the earlier waves' sums
  }
  __syncthreads();
  if (tid < kRadix) {
    uint32_t before = 0u;
    for (int w = 0; w < wave; ++w) before += lds.wsum[w];
    lds.tstart[tid] += before;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kBSortItems; ++i) {
    const uint32_t dig = (uint32_t)(key[i] >> shift) & 0xffu;
    pos[i] = lds.tstart[dig] + lds.wcnt[wave][dig] + rank[i];
  }
}

__device__ __forceinline__ void emit_point(const SegInfo& sg, int64_t pos, uint32_t p,
                                           const double* __restrict__ x,
                                           const double* __restrict__ y, int64_t SN,
                                           double* __restrict__ zs, uint32_t* __restrict__ ids) {
  const double z = seg_point(sg, x, y, p);
  uint32_t code = (int64_t)p < sg.N ? (uint32_t)(sg.y_off + p)
                                    : (uint32_t)(SN + sg.x_off + ((int64_t)p - sg.N));
  if (pos == sg.base) code |= kSegStart;
  zs[pos] = z;
  ids[pos] = code;
}

__global__ __launch_bounds__(kBSortThreads) void k_bucket_sort(
    const SegInfo* __restrict__ seg, const BucketInfo* __restrict__ buckets,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ lo,
    const double* __restrict__ hi, const uint32_t* __restrict__ bstart,
    const uint32_t* __restrict__ bsize, const uint32_t* __restrict__ ids_tmp,
    const double* __restrict__ z_tmp, uint64_t* q0,
    uint64_t* q1, uint32_t* i0, uint32_t* i1, double s_allow, int64_t SN,
    double* __restrict__ zs, uint32_t* __restrict__ ids, uint32_t* __restrict__ status) {
  __shared__ RankLds rl;
  __shared__ uint64_t stage[kBucketMax];
  __shared__ uint64_t red[kBSortThreads / kWave];
  __shared__ uint32_t dbase[kRadix], running[kRadix];
  const BucketInfo bi = buckets[blockIdx.x];
  const SegInfo sg = seg[bi.seg];
  const uint32_t n = bsize[sg.bucket0 + bi.idx];
  if (n == 0u) return;
  const int64_t off = sg.base + bstart[sg.bucket0 + bi.idx];
  const double l = lo[bi.seg], h = hi[bi.seg];
  const double qs = qscale(l, h);
  const int low_bits = resolution_bits(l, h, s_allow);
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  constexpr int W = kBSortThreads / kWave;
  const uint32_t Pb = (uint32_t)(sg.M + sg.N);
  // A merged index read back from the split is below Pb unless the split went
  // wrong; it is then clamped (no access outside the transform) and reported.
  auto checked = [&](uint32_t p) -> uint32_t {
    if (p < Pb) return p;
    atomicOr(status, kStatusInternal);
    return Pb - 1u;
  };

  auto item_index = [&](int i) { return wave * (kBSortItems * kWave) + i * kWave + lane; };

  // Bits in which the bucket's keys differ from its first key.
  auto varying_digits = [&](uint64_t v) -> uint64_t {
    for (int o = kWave / 2; o >= 1; o >>= 1) v |= __shfl_xor(v, o, kWave);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    uint64_t all = 0ull;
    for (int w = 0; w < W; ++w) all |= red[w];
    __syncthreads();
    return all;
  };
  auto needs_pass = [&](uint64_t diff, int d) {
    return ((diff >> (8 * d)) & 0xffull) != 0ull && 8 * d + 8 > low_bits;
  };

  if (n <= (uint32_t)kBucketMax) {
    // The split left the bucket's merged indices and coordinates side by side
    // (contiguous loads); the passes sort each key with its index inside the
    // bucket, and the coordinate and code of every sorted point are read back
    // from the bucket's own arrays.
    uint64_t key[kBSortItems];
    uint32_t id[kBSortItems];   // position inside the bucket
    bool valid[kBSortItems];
    double zk[kBSortItems];
#pragma unroll
    for (int i = 0; i < kBSortItems; ++i) {
      const int it = item_index(i);
      valid[i] = it < (int)n;
      id[i] = (uint32_t)it;
      zk[i] = valid[i] ? z_tmp[off + it] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kBSortItems; ++i)
      key[i] = valid[i] ? quant_key(zk[i], sg.scale, l, qs) : 0ull;
    const bool wave_active = wave * (kBSortItems * kWave) < (int)n;
    const uint64_t first = quant_key(z_tmp[off], sg.scale, l, qs);
    uint64_t diff = 0ull;
#pragma unroll
    for (int i = 0; i < kBSortItems; ++i) diff |= valid[i] ? (key[i] ^ first) : 0ull;
    diff = varying_digits(diff);
    uint32_t* sid = (uint32_t*)stage;
    for (int d = 0; d < 8; ++d) {
      if (!needs_pass(diff, d)) continue;
      uint32_t pos[kBSortItems];
      block_rank(key, valid, 8 * d, wave_active, pos, rl);
#pragma unroll
      for (int i = 0; i < kBSortItems; ++i)
        if (valid[i]) stage[pos[i]] = key[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kBSortItems; ++i) {
        const int it = item_index(i);
        key[i] = valid[i] ? stage[it] : 0ull;
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kBSortItems; ++i)
        if (valid[i]) sid[pos[i]] = id[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kBSortItems; ++i) {
        const int it = item_index(i);
        id[i] = valid[i] ? sid[it] : 0u;
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < kBSortItems; ++i) {
      if (!valid[i]) continue;
      const uint32_t local = id[i] < n ? id[i] : n - 1u;
      const uint32_t p = checked(ids_tmp[off + local]);
      uint32_t code = (int64_t)p < sg.N ? (uint32_t)(sg.y_off + p)
                                        : (uint32_t)(SN + sg.x_off + ((int64_t)p - sg.N));
      const int64_t pos = off + item_index(i);
      if (pos == sg.base) code |= kSegStart;
      zs[pos] = z_tmp[off + local];
      ids[pos] = code;
    }
    return;
  }

  // Bucket larger than the LDS: the same passes through global memory, tile
  // by tile in order (stable), with digit bases from a full histogram.
  uint64_t diff = 0ull;
  {
    const uint64_t first = point_key(sg, x, y, checked(ids_tmp[off]), l, qs);
    for (uint32_t it = tid; it < n; it += kBSortThreads) {
      const uint32_t p = checked(ids_tmp[off + it]);
      const uint64_t k = point_key(sg, x, y, p, l, qs);
      q0[off + it] = k;
      i0[off + it] = p;
      diff |= k ^ first;
    }
    diff = varying_digits(diff);
  }
  int cur = 0;
  for (int d = 0; d < 8; ++d) {
    if (!needs_pass(diff, d)) continue;
    const uint64_t* qa = cur ? q1 : q0;
    const uint32_t* ia = cur ? i1 : i0;
    uint64_t* qb = cur ? q0 : q1;
    uint32_t* ib = cur ? i0 : i1;
    if (tid < kRadix) {
      dbase[tid] = 0u;
      running[tid] = 0u;
    }
    __syncthreads();
    for (uint32_t it = tid; it < n; it += kBSortThreads)
      atomicAdd(&dbase[(uint32_t)(qa[off + it] >> (8 * d)) & 0xffu], 1u);
    __syncthreads();
    if (tid == 0) {
      uint32_t run = 0u;
      for (int b = 0; b < kRadix; ++b) {
        const uint32_t c = dbase[b];
        dbase[b] = run;
        run += c;
      }
    }
    __syncthreads();
    for (uint32_t t0 = 0; t0 < n; t0 += kBucketMax) {
      uint64_t key[kBSortItems];
      uint32_t id[kBSortItems];
      bool valid[kBSortItems];
#pragma unroll
      for (int i = 0; i < kBSortItems; ++i) {
        const uint32_t it = t0 + (uint32_t)item_index(i);
        valid[i] = it < n;
        key[i] = valid[i] ? qa[off + it] : 0ull;
        id[i] = valid[i] ? ia[off + it] : 0u;
      }
      uint32_t pos[kBSortItems];
      block_rank(key, valid, 8 * d, t0 + (uint32_t)item_index(0) - lane < n, pos, rl);
#pragma unroll
      for (int i = 0; i < kBSortItems; ++i) {
        if (!valid[i]) continue;
        const uint32_t dig = (uint32_t)(key[i] >> (8 * d)) & 0xffu;
        const uint32_t out = dbase[dig] + running[dig] + (pos[i] - rl.tstart[dig]);
        if (out < n) {
          qb[off + out] = key[i];
          ib[off + out] = id[i];
        }
      }
      __syncthreads();
      if (tid < kRadix) running[tid] += rl.thist[tid];
      __syncthreads();
    }
    cur ^= 1;
  }
  const uint32_t* ifin = cur ? i1 : i0;
  for (uint32_t it = tid; it < n; it += kBSortThreads)
    emit_point(sg, off + it, checked(ifin[off + it]), x, y, SN, zs, ids);
}

// ---------------------------------------------------------------------------
// Scan kernel (REDUCE: tile maps; otherwise the final sweeps).
// Lane layout: lane = 16 * cw + c, wave w; chunk = 4 w + cw holds kBChunkPts
// consecutive points of the tile, c is the column inside the column group
// blockIdx.y.
// ---------------------------------------------------------------------------
// Position of tile point e in the exponential table: one spare entry per
// chunk staggers the chunks read together by a wave across LDS banks.
template <int CH>
__device__ __forceinline__ int expad(int e) { return e + e / CH; }

template <int NM, bool REDUCE, int CH>
__global__ __launch_bounds__(kBThreads) void k_bscan(
    const double* __restrict__ zs, const uint32_t* __restrict__ ids, int64_t P, int64_t SN,
    int64_t SM, int R, Modes md, const int64_t* __restrict__ ne_base,
    const double* __restrict__ ne_scale, int64_t K, const double* __restrict__ alpha,
    const double* __restrict__ carry, double* __restrict__ u, double* __restrict__ tile_a,
    double* __restrict__ tile_fg) {
  constexpr int kWaves = kBThreads / kWave;
  constexpr int kCW = kWave / kBCols;   // chunks per wave (4)
  constexpr int TILE = (kBThreads / kBCols) * CH;   // points per tile
  static_assert(TILE <= kBThreads, "at most one tile point per thread in the exponential phase");
  __shared__ int64_t s_seg0;
  __shared__ uint32_t s_wflag[kWaves];
  __shared__ double s_z[TILE + 1];
  __shared__ uint32_t s_id[TILE];
  __shared__ double s_ex[2 * (TILE + TILE / CH)];   // padded per chunk: no bank conflicts
  __shared__ double s_wt[kWaves][kBCols][6];
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int cl = lane % kBCols;
  const int cw = lane / kBCols;
  const int chunk = wave * kCW + cw;
  const int col = (int)blockIdx.y * kBCols + cl;
  const bool col_ok = col < R;
  const int64_t tile = blockIdx.x;
  const int64_t t0 = tile * TILE;
  const uint32_t src_end = (uint32_t)SN, tgt_end = (uint32_t)(SN + SM);

  for (int e = tid; e < TILE; e += kBThreads) {
    const int64_t p = t0 + e;
    s_z[e + 1] = p < P ? zs[p] : 0.0;
    s_id[e] = p < P ? ids[p] : kPad;
  }
  if (tid == 0) {
    s_z[0] = t0 > 0 ? zs[t0 - 1] : 0.0;
    // the (non-empty) transform holding the tile's first point
    int64_t lo_i = 0, hi_i = K;
    while (hi_i - lo_i > 1) {
      const int64_t mid = (lo_i + hi_i) / 2;
      if (ne_base[mid] <= t0) lo_i = mid; else hi_i = mid;
    }
    s_seg0 = lo_i;
  }
  __syncthreads();
  // Scale of this thread's tile point: transforms starting inside the tile
  // after its first point advance the index.
  double my_scale = 1.0;
  {
    const uint32_t code = tid < TILE ? s_id[tid] : kPad;
    const bool flag = tid > 0 && code != kPad && (code & kSegStart);
    const uint64_t m = __ballot(flag);
    const uint32_t incl = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) +
                          (flag ? 1u : 0u);
    if (lane == 0) s_wflag[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    int64_t sidx = s_seg0 + incl;
    for (int w = 0; w < wave; ++w) sidx += s_wflag[w];
    if (tid < TILE) my_scale = ne_scale[sidx < K ? sidx : K - 1];
  }

  double b[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const uint32_t code = s_id[chunk * CH + j];
    const uint32_t r = code & ~kSegStart;
    b[j] = (code != kPad && r < src_end && col_ok) ? alpha[(int64_t)r * R + col] : 0.0;
  }
  double acc[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) acc[j] = 0.0;

  // The tile's scaled gaps (0 at the first point of a transform) and the
  // wave's largest gap, the same for every mode.
  constexpr int kPer = (TILE + kBThreads - 1) / kBThreads;
  double dz[kPer];
  bool cut[kPer];
  double dmax = 0.0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = tid + q * kBThreads;
    const uint32_t code = e < TILE ? s_id[e] : kPad;
    cut[q] = code != kPad && (code & kSegStart);
    dz[q] = (code == kPad || cut[q]) ? 0.0 : (s_z[e + 1] - s_z[e]) * my_scale;
    dmax = fmax(dmax, fabs(dz[q]));
  }
  for (int o = kWave / 2; o >= 1; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, kWave));

#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    // Mode exponentials of the tile's gaps, 0 at the first point of a transform.
    {
      const double rr = md.tau_abs[k] * dmax;
      int D = kTaylorMax;
#pragma unroll
      for (int d = kTaylorMax; d >= 1; --d)
        if (rr <= md.taylor_thr[d]) D = d;
      const double dz_lim = md.dz_lim[k];
      // A gap beyond the Taylor range is halved k times into it, its
      // exponential taken there and squared k times
      // (exp(-tau dz) = exp(-tau dz / 2^k)^(2^k)): the relative error grows to
      // about 2^k u, but |exp(-tau dz)| = exp(-Re(tau) dz) falls faster, so the
      // absolute error stays at the rounding level.
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        double d = dz[q];
        int halvings = 0;
        while (fabs(d) > dz_lim && halvings < 1100) {
          d *= 0.5;
          ++halvings;
        }
        // One degree for the wave (the full one if any lane halved), so the
        // coefficients are uniform loads and the polynomial is unrolled.
        const int Dw = __ballot(halvings != 0) ? kTaylorMax : D;
        C<double> ex = {0.0, 0.0};
#pragma unroll
        for (int m = kTaylorMax; m >= 0; --m) {
          if (m <= Dw) {
            ex.re = fma(ex.re, d, md.coef_re[k][m]);
            ex.im = fma(ex.im, d, md.coef_im[k][m]);
          }
        }
        for (int h = 0; h < halvings; ++h) ex = cmul(ex, ex);
        if (cut[q]) ex = {0.0, 0.0};
        const int e = tid + q * kBThreads;
        if (e < TILE) {
          s_ex[2 * expad<CH>(e)] = ex.re;
          s_ex[2 * expad<CH>(e) + 1] = ex.im;
        }
      }
    }
    __syncthreads();

    // Chunk map: A = prod e, F = sum_q b_q prod_{p > q} e_p, G = sum_q b_q prod_{p <= q} e_p.
    Seg<double> s;
    {
      C<double> a = {1.0, 0.0}, f = {0.0, 0.0}, g = {0.0, 0.0};
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int e = chunk * CH + j;
        const C<double> ex = {s_ex[2 * expad<CH>(e)], s_ex[2 * expad<CH>(e) + 1]};
        a = cmul(a, ex);
        f = cfma(ex, f, C<double>{b[j], 0.0});
        g.re = fma(b[j], a.re, g.re);
        g.im = fma(b[j], a.im, g.im);
      }
      s.a = a;
      s.f = f;
      s.g = g;
    }
    // Scans over the wave's chunks of the same column (lanes 16 apart).
    Seg<double> pf = s, sb = s;
#pragma unroll
    for (int o = kBCols; o < kWave; o <<= 1) {
      Seg<double> l, r;
      l.a.re = shfl_up(pf.a.re, o); l.a.im = shfl_up(pf.a.im, o);
      l.f.re = shfl_up(pf.f.re, o); l.f.im = shfl_up(pf.f.im, o);
      if (lane >= o) {
        pf.f = cfma(pf.a, l.f, pf.f);
        pf.a = cmul(l.a, pf.a);
      }
      r.a.re = shfl_down(sb.a.re, o); r.a.im = shfl_down(sb.a.im, o);
      r.g.re = shfl_down(sb.g.re, o); r.g.im = shfl_down(sb.g.im, o);
      if (lane + o < kWave) {
        sb.g = cfma(sb.a, r.g, sb.g);
        sb.a = cmul(sb.a, r.a);
      }
    }
    if (cw == kCW - 1) {
      s_wt[wave][cl][0] = pf.a.re; s_wt[wave][cl][1] = pf.a.im;
      s_wt[wave][cl][2] = pf.f.re; s_wt[wave][cl][3] = pf.f.im;
    }
    if (cw == 0) {
      s_wt[wave][cl][4] = sb.g.re; s_wt[wave][cl][5] = sb.g.im;
    }
    __syncthreads();

    if (REDUCE) {
      if (tid < kBCols) {
        Seg<double> t = seg_identity<double>();
        for (int w = 0; w < kWaves; ++w) {
          const double* v = s_wt[w][tid];
          t = compose(t, Seg<double>{{v[0], v[1]}, {v[2], v[3]}, {v[4], v[5]}});
        }
        const int c2 = (int)blockIdx.y * kBCols + tid;
        if (tid == 0 && blockIdx.y == 0) {
          double* o = tile_a + ((size_t)tile * NM + k) * 2;
          o[0] = t.a.re;
          o[1] = t.a.im;
        }
        if (c2 < R) {
          double* o = tile_fg + (((size_t)tile * NM + k) * R + c2) * 4;
          o[0] = t.f.re; o[1] = t.f.im;
          o[2] = t.g.re; o[3] = t.g.im;
        }
      }
    } else {
      C<double> cf = {0.0, 0.0}, cb = {0.0, 0.0};
      if (col_ok) {
        const double* c = carry + (((size_t)tile * NM + k) * R + col) * 4;
        cf = {c[0], c[1]};
        cb = {c[2], c[3]};
      }
      for (int w = 0; w < wave; ++w) {
        const double* v = s_wt[w][cl];
        cf = cfma(C<double>{v[0], v[1]}, cf, C<double>{v[2], v[3]});
      }
      for (int w = kWaves - 1; w > wave; --w) {
        const double* v = s_wt[w][cl];
        cb = cfma(C<double>{v[0], v[1]}, cb, C<double>{v[4], v[5]});
      }
      Seg<double> xl, xr;
      xl.a.re = shfl_up(pf.a.re, kBCols); xl.a.im = shfl_up(pf.a.im, kBCols);
      xl.f.re = shfl_up(pf.f.re, kBCols); xl.f.im = shfl_up(pf.f.im, kBCols);
      xr.a.re = shfl_down(sb.a.re, kBCols); xr.a.im = shfl_down(sb.a.im, kBCols);
      xr.g.re = shfl_down(sb.g.re, kBCols); xr.g.im = shfl_down(sb.g.im, kBCols);
      if (cw > 0) cf = cfma(xl.a, cf, xl.f);
      if (cw < kCW - 1) cb = cfma(xr.a, cb, xr.g);

      const double om_re = md.om_re[k], om_im = md.om_im[k];
      // Both sweeps in one loop (forward step j, backward step CH-1-j): the two
      // chains of dependent complex FMAs are independent and interleave.
      C<double> hh = cf, g = cb;
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int jb = CH - 1 - j;
        const int e = chunk * CH + j, eb = chunk * CH + jb;
        const C<double> ex = {s_ex[2 * expad<CH>(e)], s_ex[2 * expad<CH>(e) + 1]};
        const C<double> exb = {s_ex[2 * expad<CH>(eb)], s_ex[2 * expad<CH>(eb) + 1]};
        hh = cfma(ex, hh, C<double>{b[j], 0.0});
        acc[j] = fma(om_re, hh.re, fma(-om_im, hh.im, acc[j]));
        acc[jb] = fma(om_re, g.re, fma(-om_im, g.im, acc[jb]));
        g = cmul(exb, cadd(g, C<double>{b[jb], 0.0}));
      }
    }
    __syncthreads();   // s_ex and s_wt are rewritten for the next mode
  }

  if (!REDUCE && col_ok) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const uint32_t code = s_id[chunk * CH + j];
      const uint32_t r = code & ~kSegStart;
      if (code != kPad && r >= src_end && r < tgt_end) u[(int64_t)(r - src_end) * R + col] = acc[j];
    }
  }
}

template <int NM, int CH>
hipError_t batch_scan(const BatchDims& d, const Modes& md, const int64_t* ne_base,
                      const double* ne_scale, const double* alpha, double* u, const BatchWork& w,
                      hipStream_t s) {
  constexpr int TILE = (kBThreads / kBCols) * CH;
  const int64_t tiles = (d.P + TILE - 1) / TILE;
  const dim3 grid((unsigned)tiles, (unsigned)((d.R + kBCols - 1) / kBCols));
  hipLaunchKernelGGL((k_bscan<NM, true, CH>), grid, dim3(kBThreads), 0, s, w.zs, w.ids, d.P, d.SN,
                     d.SM, d.R, md, ne_base, ne_scale, d.K, alpha, (const double*)nullptr,
                     (double*)nullptr, w.tile_a, w.tile_fg);
  const int nq = NM * d.R;
  hipError_t e = launch_carries<double>(BatchMaps<double>{w.tile_a, w.tile_fg, NM, d.R}, tiles,
                                        nq, w.chunk_agg, w.chunk_carry, w.carry, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_bscan<NM, false, CH>), grid, dim3(kBThreads), 0, s, w.zs, w.ids, d.P, d.SN,
                     d.SM, d.R, md, ne_base, ne_scale, d.K, alpha, (const double*)w.carry, u,
                     (double*)nullptr, (double*)nullptr);
  return hipGetLastError();
}

template <int NM>
hipError_t batch_scan_chunk(int chunk, const BatchDims& d, const Modes& md, const int64_t* ne_base,
                            const double* ne_scale, const double* alpha, double* u,
                            const BatchWork& w, hipStream_t s) {
  return chunk == 8 ? batch_scan<NM, 8>(d, md, ne_base, ne_scale, alpha, u, w, s)
                    : batch_scan<NM, 16>(d, md, ne_base, ne_scale, alpha, u, w, s);
}

__global__ void k_clear_words(uint32_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Sorted codes (transform-start flag cleared) and coordinates of a batch.
__global__ __launch_bounds__(256) void k_batch_sorted(const uint32_t* __restrict__ ids,
                                                      const double* __restrict__ zs, int64_t P,
                                                      uint32_t* __restrict__ codes,
                                                      double* __restrict__ z) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += stride) {
    if (codes) codes[p] = ids[p] & ~kSegStart;
    if (z) z[p] = zs[p];
  }
}

}  // namespace

BatchWork batch_layout(void* base, const BatchDims& d) {
  BatchWork w;
  memset(&w, 0, sizeof(w));
  char* b = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? (void*)(b + off) : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  const size_t P = (size_t)(d.P > 0 ? d.P : 1);
  const int64_t chunks = (d.tiles + kWave - 1) / kWave;
  const size_t nq = (size_t)d.n_modes * (size_t)d.R;
  w.status = (uint32_t*)take(sizeof(uint32_t) * 64);
  w.lo = (double*)take(sizeof(double) * (size_t)d.B);
  w.hi = (double*)take(sizeof(double) * (size_t)d.B);
  w.counts = (uint32_t*)take(sizeof(uint32_t) * (size_t)(d.n_counts > 0 ? d.n_counts : 1));
  w.offs = (uint32_t*)take(sizeof(uint32_t) * (size_t)(d.n_counts > 0 ? d.n_counts : 1));
  w.bstart = (uint32_t*)take(sizeof(uint32_t) * (size_t)d.n_buckets);
  w.bsize = (uint32_t*)take(sizeof(uint32_t) * (size_t)d.n_buckets);
  w.ids_tmp = (uint32_t*)take(sizeof(uint32_t) * P);
  w.z_tmp = (double*)take(sizeof(double) * P);
  w.qbuf[0] = (uint64_t*)take(sizeof(uint64_t) * P);
  w.qbuf[1] = (uint64_t*)take(sizeof(uint64_t) * P);
  w.ibuf[0] = (uint32_t*)take(sizeof(uint32_t) * P);
  w.ibuf[1] = (uint32_t*)take(sizeof(uint32_t) * P);
  w.zs = (double*)take(sizeof(double) * P);
  w.ids = (uint32_t*)take(sizeof(uint32_t) * P);
  w.tile_a = (double*)take(sizeof(double) * 2 * (size_t)d.n_modes * (size_t)d.tiles);
  w.tile_fg = (double*)take(sizeof(double) * 4 * nq * (size_t)d.tiles);
  w.chunk_agg = (double*)take(sizeof(double) * 6 * nq * (size_t)chunks);
  w.chunk_carry = (double*)take(sizeof(double) * 4 * nq * (size_t)chunks);
  w.carry = (double*)take(sizeof(double) * 4 * nq * (size_t)d.tiles);
  w.total = off;
  return w;
}

hipError_t batch_eval_launch(const BatchDims& d, const BatchTables& t, const Modes& md,
                             double s_allow, int chunk, const double* x, const double* y,
                             const double* alpha, double* u, const BatchWork& w, hipStream_t s) {
  const SegInfo* seg = t.seg;
  const ChunkInfo* chunks = t.chunks;
  const BucketInfo* buckets = t.buckets;
  const int64_t* ne_base = t.ne_base;
  const double* ne_scale = t.ne_scale;
  const int max_nb_log2 = t.max_nb_log2;
  hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, s, w.status, 64);
  if (d.P == 0) return hipGetLastError();
  hipLaunchKernelGGL(k_seg_minmax, dim3((unsigned)d.B), dim3(256), 0, s, seg, x, y, w.lo, w.hi,
                     w.status);
  const size_t nb_max = (size_t)1 << max_nb_log2;
  if (d.n_chunks > 0) {
    hipLaunchKernelGGL(k_seg_count, dim3((unsigned)d.n_chunks), dim3(256), nb_max * sizeof(uint32_t),
                       s, seg, chunks, x, y, (const double*)w.lo, (const double*)w.hi, w.counts);
  }
  hipLaunchKernelGGL(k_seg_offsets, dim3((unsigned)d.B), dim3(256), 0, s, seg,
                     (const uint32_t*)w.counts, w.offs, w.bstart, w.bsize);
  if (d.n_chunks > 0) {
    hipLaunchKernelGGL(k_seg_scatter, dim3((unsigned)d.n_chunks), dim3(256),
                       4 * nb_max * sizeof(uint32_t), s, seg, chunks, x, y, (const double*)w.lo,
                       (const double*)w.hi, (const uint32_t*)w.offs, w.ids_tmp, w.z_tmp);
  }
  hipLaunchKernelGGL(k_bucket_sort, dim3((unsigned)t.n_buckets), dim3(kBSortThreads), 0, s, seg,
                     buckets, x, y, (const double*)w.lo, (const double*)w.hi,
                     (const uint32_t*)w.bstart, (const uint32_t*)w.bsize,
                     (const uint32_t*)w.ids_tmp, (const double*)w.z_tmp, w.qbuf[0], w.qbuf[1],
                     w.ibuf[0], w.ibuf[1],
                     s_allow, d.SN, w.zs, w.ids, w.status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (md.n) {
    case 1: return batch_scan_chunk<1>(chunk, d, md, ne_base, ne_scale, alpha, u, w, s);
    case 2: return batch_scan_chunk<2>(chunk, d, md, ne_base, ne_scale, alpha, u, w, s);
    case 3: return batch_scan_chunk<3>(chunk, d, md, ne_base, ne_scale, alpha, u, w, s);
    case 4: return batch_scan_chunk<4>(chunk, d, md, ne_base, ne_scale, alpha, u, w, s);
    case 5: return batch_scan_chunk<5>(chunk, d, md, ne_base, ne_scale, alpha, u, w, s);
    case 6: return batch_scan_chunk<6>(chunk, d, md, ne_base, ne_scale, alpha, u, w, s);
    case 7: return batch_scan_chunk<7>(chunk, d, md, ne_base, ne_scale, alpha, u, w, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t batch_sorted_copy(const BatchDims& d, const BatchWork& w, uint32_t* codes, double* z,
                             hipStream_t s) {
  if (d.P == 0 || (!codes && !z)) return hipSuccess;
  int64_t blocks = (d.P + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_batch_sorted, dim3((unsigned)blocks), dim3(256), 0, s, w.ids, w.zs, d.P,
                     codes, z);
  return hipGetLastError();
}

}  // namespace fgt
