// Stable LSD radix sort of the merged point set [y_1..y_N, x_1..x_M] on gfx950.
//
// The paper sorts targets and sources in ascending order before the
// recurrences (Section 4) and times that step separately (Tables 1-2).  Here
// both sets are sorted together as order-preserving unsigned keys (FP64: the
// grid code of Codec<double>, else IEEE order keys) with a 32-bit payload p
// (p < N: source p, else target p - N).  Stability places a source before a
// target with the same coordinate, which realises the "y_j <= x_i belongs to
// h+" split of (4.4).
//
// Kernels, all on the caller's stream:
//   k_clear       zero histograms, tile counters, status word, look-back[0]
//   k_range       (FP64) smallest and largest coordinate, their finest
//                 power-of-two granularity, non-finite flag
//   k_histogram   one read of the coordinates: the histograms of all digits
//                 above the sort resolution at once (FP32: all digits, and the
//                 range and the non-finite flag)
//   k_plan        the FP64 key code for the range; per pass: does the digit
//                 vary?  where does the pass read from and write to?
//                 exclusive digit offsets
//   k_onesweep    one pass per digit: stable in-tile ranking with wave ballots,
//                 tile offsets by decoupled look-back (Merrill & Garland),
//                 scatter staged through LDS so writes are coalesced runs.
//                 Passes whose digit is constant return at once.  The last
//                 pass stores the decoded coordinates and the final ids (the
//                 scan's tile reduce gathers the strengths by id).
#include "fgt_internal.h"

namespace fgt {
namespace {

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
constexpr int kRaw = 2;
// A look-back wait longer than this means a predecessor tile never published;
// the pass then stops waiting and raises kStatusInternal instead of hanging.
constexpr uint32_t kSpinLimit = 1u << 24;
constexpr int kLookWindow = 4;   // predecessors read per look-back step

__global__ void k_clear(uint32_t* __restrict__ p, size_t n_words) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n_words; i += stride) p[i] = 0u;
}

// Visits every coordinate once, y[0..N) then x[0..P-N), grid-strided, with
// 16-byte loads where an array is 16-byte aligned (two FP64 or four FP32
// coordinates per load; kBatch loads issued together before any is used) and
// single loads otherwise or for the tail.
template <class T, int kBatch, class F>
__device__ __forceinline__ void visit_points(const T* __restrict__ x, const T* __restrict__ y,
                                             int64_t N, int64_t P, F f) {
  typedef T V __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int L = 16 / sizeof(T);
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int part = 0; part < 2; ++part) {
    const T* __restrict__ a = part == 0 ? y : x;
    const int64_t n = part == 0 ? N : P - N;
    if (n <= 0) continue;
    int64_t done = 0;
    if (((uintptr_t)a & 15u) == 0) {
      const int64_t nv = n / L;
      const V* __restrict__ av = reinterpret_cast<const V*>(a);
      for (int64_t p0 = gtid; p0 < nv; p0 += stride * kBatch) {
        V vb[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
          const int64_t p = p0 + i * stride;
          vb[i] = av[p < nv ? p : p0];
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
          if (p0 + i * stride >= nv) break;
#pragma unroll
          for (int l = 0; l < L; ++l) f(vb[i][l]);
        }
      }
      done = nv * L;
    }
    for (int64_t p0 = done + gtid; p0 < n; p0 += stride * kBatch) {
      T zb[kBatch];
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        const int64_t p = p0 + i * stride;
        zb[i] = a[p < n ? p : p0];
      }
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        if (p0 + i * stride >= n) break;
        f(zb[i]);
      }
    }
  }
}

// Smallest and largest IEEE order key of a thread's points, and whether any
// is not finite; folded over the block and published with two atomics per
// block (the smallest as the largest complement, so that zeroed words start
// both).  publish() is called by every thread of the block.
struct RangeAcc {
  uint64_t kmin = ~0ull, kmax = 0ull;
  uint32_t gran = 0u;   // 2048 - the finest granularity exponent seen (FP64), 0 if none
  bool bad = false;
  template <class T>
  __device__ __forceinline__ void add(T z) {
    const uint64_t k = (uint64_t)to_key(z);
    kmin = k < kmin ? k : kmin;
    kmax = k > kmax ? k : kmax;
    bad |= !isfinite(z);
    if constexpr (sizeof(T) == 8) {
      const uint32_t gv = (z != 0.0 && isfinite(z)) ? (uint32_t)(2048 - granularity_exp(z)) : 0u;
      gran = gv > gran ? gv : gran;
    }
  }
  __device__ __forceinline__ void publish(unsigned long long* range, uint32_t* status) {
    __shared__ uint64_t wmin[1024 / kWave], wmax[1024 / kWave];
    __shared__ uint32_t wgran[1024 / kWave];
    for (int o = kWave / 2; o >= 1; o >>= 1) {
      const uint64_t a = __shfl_xor(kmin, o, kWave);
      const uint64_t b = __shfl_xor(kmax, o, kWave);
      const uint32_t c = __shfl_xor(gran, o, kWave);
      kmin = a < kmin ? a : kmin;
      kmax = b > kmax ? b : kmax;
      gran = c > gran ? c : gran;
    }
    if (bad) atomicOr(status, kStatusNonFinite);
    const int wave = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0) {
      wmin[wave] = kmin;
      wmax[wave] = kmax;
      wgran[wave] = gran;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x / kWave); ++w) {
        kmin = wmin[w] < kmin ? wmin[w] : kmin;
        kmax = wmax[w] > kmax ? wmax[w] : kmax;
        gran = wgran[w] > gran ? wgran[w] : gran;
      }
      atomicMax(&range[0], (unsigned long long)~kmin);
      atomicMax(&range[1], (unsigned long long)kmax);
      if (gran) atomicMax(&range[2], (unsigned long long)gran);
    }
  }
};

template <class T>
__global__ __launch_bounds__(1024) void k_range(const T* __restrict__ x, const T* __restrict__ y,
                                               int64_t N, int64_t P,
                                               unsigned long long* __restrict__ range,
                                               uint32_t* __restrict__ status) {
  RangeAcc acc;
  if constexpr (sizeof(T) == 8) {
    // Folded as doubles (one min and one max instruction a point; -0 and +0
    // map to the same key) and converted to order keys once.  Any non-finite
    // point publishes the range [-inf, +inf]: like a NaN's key it selects IEEE
    // keys with every bit sorted.
    double lo = INFINITY, hi = -INFINITY;
    uint32_t gran = 0u;
    bool bad = false;
    visit_points<T, 8>(x, y, N, P, [&](T z) {
      lo = fmin(lo, z);
      hi = fmax(hi, z);
      const bool fin = isfinite(z);
      bad |= !fin;
      const uint32_t gv = (z != 0.0 && fin) ? (uint32_t)(2048 - granularity_exp(z)) : 0u;
      gran = gv > gran ? gv : gran;
    });
    acc.kmin = bad ? to_key(-INFINITY) : to_key(lo);
    acc.kmax = bad ? to_key(INFINITY) : to_key(hi);
    acc.gran = gran;
    acc.bad = bad;
  } else {
    visit_points<T, 8>(x, y, N, P, [&](T z) { acc.add(z); });
  }
  acc.publish(range, status);
}

template <class T>
__device__ __forceinline__ Codec<T> codec_from_range(const unsigned long long* range,
                                                     double code_tol) {
  if constexpr (sizeof(T) == 8) {
    const int gran = range[2] ? 2048 - (int)range[2] : 1 << 20;
    return make_codec(~(uint64_t)range[0], (uint64_t)range[1], gran, code_tol);
  } else {
    (void)range;
    (void)code_tol;
    return Codec<float>{};
  }
}

// Sort resolution in key bits.  Keys that agree above bit b differ by less
// than 2^b, so their coordinates by less than unit (2^b + slack): the lowest
// b bits with unit (2^b + slack) <= the resolution need not be sorted.  *top:
// the keys are below 2^top.
template <class T>
__device__ __forceinline__ int resolution_bits(const unsigned long long* range,
                                               const SortRes& res, const Codec<T>& cd, int* top) {
  double key_width = res.key_width;
  double unit;   // coordinate distance of one key step (bound)
  double slack;  // key steps that the encoding may lose
  if constexpr (sizeof(T) == 8) {
    if (cd.quant) {
      // Grid points decode exactly, others move by less than g:
      // |z1 - z2| < (|q1 - q2| + 1) g.
      unit = cd.g;
      slack = 1.0;
      key_width = res.key_width_q;
      *top = 63;
    } else {
      // IEEE order keys: the largest |z| has the widest spacing, ulp.
      const double a = from_key((uint64_t)~(uint64_t)range[0]);
      const double c = from_key((uint64_t)range[1]);
      const double zmax = fabs(a) > fabs(c) ? fabs(a) : fabs(c);
      const int ex = (int)((__double_as_longlong(zmax) >> 52) & 0x7ff);
      unit = ex == 0x7ff ? INFINITY : ldexp(1.0, (ex == 0 ? 1 : ex) - 1075);
      slack = 0.0;
      *top = 64;
    }
  } else {
    (void)cd;
    const float a = from_key((uint32_t)~(uint64_t)range[0]);
    const float c = from_key((uint32_t)range[1]);
    const float zmax = fabsf(a) > fabsf(c) ? fabsf(a) : fabsf(c);
    const int ex = (int)((__float_as_uint(zmax) >> 23) & 0xff);
    unit = ex == 0xff ? INFINITY : ldexp(1.0, (ex == 0 ? 1 : ex) - 150);
    slack = 0.0;
    *top = 32;
  }
  int lo = 0;
  if (key_width > 0.0 && unit < INFINITY)
    while (lo < *top - 1 && unit * (ldexp(1.0, lo + 1) + slack) <= key_width) ++lo;
  return lo;
}

// Digits of this sort.  FP64: the bits from the resolution to the top of the
// keys are cut into passes of 8 or 9 bits, whichever needs fewer passes (8 on
// a tie).  FP32 (whose histograms are counted while its range is still being
// gathered): four 8-bit digits from bit 0, of which k_plan skips the ones
// below the resolution.
struct DigitLayout {
  int lo_bit;   // lowest sorted bit
  int bits;     // digit width, 8 or 9
  int passes;   // 1 .. 8
};
template <class T>
__device__ __forceinline__ DigitLayout digit_layout(const unsigned long long* range,
                                                    const SortRes& res, const Codec<T>& cd) {
  DigitLayout L{0, 8, 4};
  if constexpr (sizeof(T) == 8) {
    int top = 64;
    L.lo_bit = resolution_bits<T>(range, res, cd, &top);
    const int nb = top - L.lo_bit;
    const int p8 = (nb + 7) / 8, p9 = (nb + 8) / 9;
    L.bits = p9 < p8 ? 9 : 8;
    L.passes = p9 < p8 ? p9 : p8;
  } else {
    (void)range;
    (void)res;
    (void)cd;
  }
  return L;
}

// Histograms of every pass's digit of all keys.  FP64 keys need the range
// (k_range first), which also fixes the digit layout; FP32 keys are plain IEEE
// order keys and the range is gathered here.
template <class T>
__global__ __launch_bounds__(256) void k_histogram(const T* __restrict__ x, const T* __restrict__ y,
                                                   int64_t N, int64_t P,
                                                   uint32_t* __restrict__ hist,
                                                   uint32_t* __restrict__ status,
                                                   unsigned long long* __restrict__ range,
                                                   SortRes res) {
  using K = typename KeyOf<T>::type;
  constexpr int D = KeyOf<T>::kDigits;
  constexpr bool kGatherRange = sizeof(T) == 4;
  __shared__ uint32_t h[D * kSortRadix];
  for (int i = threadIdx.x; i < D * kSortRadix; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const Codec<T> cd = codec_from_range<T>(range, res.code_tol);
  const DigitLayout L = digit_layout<T>(range, res, cd);
  const uint32_t mask = (1u << L.bits) - 1u;

  RangeAcc acc;
  visit_points<T, 8>(x, y, N, P, [&](T z) {
    if (kGatherRange) acc.add(z);
    const K k = cd.encode(z);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (d >= L.passes) continue;
      const uint32_t dig = (uint32_t)(k >> (L.lo_bit + L.bits * d)) & mask;
      atomicAdd(&h[d * kSortRadix + dig], 1u);
    }
  });
  if (kGatherRange) acc.publish(range, status);
  __syncthreads();
  for (int i = threadIdx.x; i < D * kSortRadix; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// One block of 8 waves: wave d scans digit d's counts (kSortRadix / 64 per lane).
template <class T>
__global__ __launch_bounds__(512) void k_plan(const uint32_t* __restrict__ hist, int64_t P,
                                              const unsigned long long* __restrict__ range,
                                              SortRes res, uint32_t* __restrict__ dig_off,
                                              PassInfo* __restrict__ pass) {
  constexpr int D = KeyOf<T>::kDigits;
  __shared__ int trivial[8];
  const int b = threadIdx.x;
  const int wave = b / kWave, lane = b % kWave;
  if (b < 8) trivial[b] = 0;
  __syncthreads();
  if (wave < D) {
    constexpr int kPer = kSortRadix / kWave;   // consecutive digit values per lane
    const uint32_t* h = hist + wave * kSortRadix + kPer * lane;
    uint32_t c[kPer];
    uint32_t own = 0u;
    bool full = false;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      c[q] = h[q];
      own += c[q];
      full |= (int64_t)c[q] == P;
    }
    if (full) trivial[wave] = 1;
    uint32_t incl = own;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t v = __shfl_up(incl, (unsigned)o, kWave);
      if (lane >= o) incl += v;
    }
    uint32_t* out = dig_off + wave * kSortRadix + kPer * lane;
    uint32_t e = incl - own;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      out[q] = e;
      e += c[q];
    }
  }
  __syncthreads();
  if (b == 0) {
    const Codec<T> cd = codec_from_range<T>(range, res.code_tol);
    if constexpr (sizeof(T) == 8) {
      pass->code_quant = cd.quant;
      pass->code_F = cd.F;
      pass->code_L = cd.L;
      pass->code_g = cd.g;
      pass->code_inv_g = cd.inv_g;
    }
    const DigitLayout L = digit_layout<T>(range, res, cd);
    // FP32: whole 8-bit digits below the resolution are left unsorted.
    int skip = 0;
    if constexpr (sizeof(T) == 4) {
      int top = 32;
      skip = resolution_bits<T>(range, res, cd, &top) / 8;
    }
    for (int d = 0; d < skip; ++d) trivial[d] = 1;
    pass->skipped_low = L.lo_bit + 8 * skip;
    pass->bits = L.bits;
    int any = 0;
    for (int d = 0; d < L.passes; ++d) any |= !trivial[d];
    int runs = 0, last_out = 0, last_pass = 0;
    for (int d = 0; d < 8; ++d) {
      int run = d < L.passes && !trivial[d];
      if (!any && d == L.passes - 1) run = 1;  // all keys equal: one pass materialises them
      pass->run[d] = run;
      pass->shift[d] = L.lo_bit + L.bits * d;
      if (run) {
        pass->src[d] = runs == 0 ? kRaw : (runs - 1) % 2;
        last_out = runs % 2;
        last_pass = d;
        ++runs;
      } else {
        pass->src[d] = -1;
      }
    }
    pass->final_buf = last_out;
    pass->last_pass = last_pass;
  }
}

// LDS of one radix tile.
template <class T>
struct SweepLds {
  // Per-wave running digit counts, then each wave's first slot per digit in
  // the tile's digit order (tile-local digit start + earlier waves' counts).
  uint16_t wcnt[kSortWaves][kSortRadix];
  // Output position of a digit's run minus its tile-local start: key j of the
  // digit-sorted tile goes to goff[digit] + j.
  uint32_t goff[kSortRadix];
  uint32_t wsum[kSortRadix / kWave];
  uint32_t thist[kSortRadix];                     // tile digit histogram
  typename KeyOf<T>::type stage[kSortTile];       // keys, then (reused) payloads, in digit order
};

// One tile of a radix pass.  kFull: the tile holds kSortTile points (every
// tile but the last), so no item needs a bounds check.  The last tile's loads
// read a clamped, in-bounds index and mask the value: no branch per item.
template <class T, bool kFull>
__device__ __forceinline__ void sweep_tile(
    SweepLds<T>& lds, int tile, int d, const T* __restrict__ x, const T* __restrict__ y,
    int64_t N, int64_t P, void* keys0, void* keys1, uint32_t* idx0, uint32_t* idx1,
    uint32_t* __restrict__ ids_out, const uint32_t* __restrict__ dig_off,
    const PassInfo* __restrict__ pass, uint64_t* lb_cur, uint32_t* __restrict__ status) {
  using K = typename KeyOf<T>::type;
  auto& wcnt = lds.wcnt;
  auto& goff = lds.goff;
  auto& wsum = lds.wsum;
  auto& thist = lds.thist;
  auto& stage = lds.stage;
  const int tid = threadIdx.x;
  const int src = pass->src[d];
  const int dbits = pass->bits;          // 8 or 9 for the whole sort
  const int ndig = 1 << dbits;
  const bool digit_thread = tid < ndig;   // threads 0..ndig-1 own one digit value each

  const K* kin = src == 1 ? (const K*)keys1 : (const K*)keys0;
  const uint32_t* iin = src == 1 ? idx1 : idx0;
  K* kout = src == 0 ? (K*)keys1 : (K*)keys0;
  uint32_t* iout = src == 0 ? idx1 : idx0;

  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int shift = pass->shift[d];
  const uint32_t mask = (uint32_t)ndig - 1u;
  const int64_t base = (int64_t)tile * kSortTile + (int64_t)wave * (kSortItems * kWave);

  K key[kSortItems];
  uint32_t id[kSortItems];
  uint32_t rank[kSortItems];
  // Separate load loops (the source is the same for the whole pass), each
  // issuing all of its loads before any is used.  The points of the first pass
  // and the keys of the middle passes are read once: nontemporal loads keep
  // them from displacing the lines in which the scattered runs of the pass are
  // being written.  The last pass loads normally (nontemporal measured slower
  // there).
  if (src == kRaw) {
    T z[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const int64_t p = base + i * kWave + lane;
      const int64_t pc = (kFull || p < P) ? p : P - 1;   // in bounds; masked below
      z[i] = pc < N ? __builtin_nontemporal_load(&y[pc]) : __builtin_nontemporal_load(&x[pc - N]);
      id[i] = (kFull || p < P) ? (uint32_t)p : 0u;
    }
    const Codec<T> cd = codec_of<T>(pass);
#pragma unroll
    for (int i = 0; i < kSortItems; ++i)
      key[i] = (kFull || base + i * kWave + lane < P) ? cd.encode(z[i]) : (K)0;
  } else if (d == pass->last_pass) {
    // The empty asm keeps the compiler from merging this loop with the one
    // below, which would drop the nontemporal hint of the middle passes.
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const int64_t p = base + i * kWave + lane;
      const int64_t pc = (kFull || p < P) ? p : P - 1;
      const K kv = kin[pc];
      const uint32_t iv = iin[pc];
      key[i] = (kFull || p < P) ? kv : (K)0;
      id[i] = (kFull || p < P) ? iv : 0u;
    }
    asm volatile("" ::: "memory");
  } else {
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const int64_t p = base + i * kWave + lane;
      const int64_t pc = (kFull || p < P) ? p : P - 1;
      const K kv = __builtin_nontemporal_load(&kin[pc]);
      const uint32_t iv = __builtin_nontemporal_load(&iin[pc]);
      key[i] = (kFull || p < P) ? kv : (K)0;
      id[i] = (kFull || p < P) ? iv : 0u;
    }
  }

  // Tile histogram first, so the tile's counts are published before the
  // (longer) stable ranking and successors waiting on them move on sooner.
#pragma unroll
  for (int i = 0; i < kSortItems; ++i)
    if (kFull || base + i * kWave + lane < P)
      atomicAdd(&thist[(uint32_t)(key[i] >> shift) & mask], 1u);
  __syncthreads();
  uint32_t tcount = 0u;
  if (digit_thread) {
    tcount = thist[tid];
    __hip_atomic_store(&lb_cur[(size_t)tile * kSortRadix + tid], kFlagAgg | (uint64_t)tcount,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  // Stable ranking inside the wave, items in order (i, lane): lanes with the
  // same digit are found with one ballot per digit bit (a lane keeps the
  // ballot's lanes where its own bit is set, the others where it is clear:
  // ballot XOR the lane's bit as a sign mask, inverted); the lowest lane of
  // each group advances the wave's running count.
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t p = base + i * kWave + lane;
    const bool valid = kFull || p < P;
    const uint32_t dig = (uint32_t)(key[i] >> shift) & mask;
    const uint64_t live = kFull ? ~0ull : __ballot(valid);
    uint32_t pl = (uint32_t)live, ph = (uint32_t)(live >> 32);
#pragma unroll
    for (int bit = 0; bit < kSortBits; ++bit) {
      if (bit < dbits) {   // uniform: the last bit only for 9-bit digits
        const int32_t m = (int32_t)(dig << (31 - bit)) >> 31;   // the lane's bit as a sign mask
        const uint64_t bal = __ballot(m < 0);
        pl &= ~((uint32_t)bal ^ (uint32_t)m);
        ph &= ~((uint32_t)(bal >> 32) ^ (uint32_t)m);
      }
    }
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(ph, __builtin_amdgcn_mbcnt_lo(pl, 0u));
    const uint32_t count = (uint32_t)__popc(pl) + (uint32_t)__popc(ph);
    const uint32_t before = wcnt[wave][dig];
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0u) wcnt[wave][dig] = (uint16_t)(before + count);
    __builtin_amdgcn_wave_barrier();
    rank[i] = before + below;
  }

  // Exclusive scan of the tile histogram over digits (thread tid owns digit tid).
  uint32_t tstart = 0u;   // the digit's tile-local start (digit threads)
  {
    uint32_t incl = tcount;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t v = __shfl_up(incl, (unsigned)o, kWave);
      if (lane >= o) incl += v;
    }
    if (digit_thread && lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    if (digit_thread) {
      uint32_t before = 0u;
      for (int w = 0; w < wave; ++w) before += wsum[w];
      tstart = before + incl - tcount;
      // running per-wave counts -> each wave's first slot (at most kSortTile)
      uint32_t run_sum = tstart;
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) {
        const uint32_t c = wcnt[w][tid];
        wcnt[w][tid] = (uint16_t)run_sum;
        run_sum += c;
      }
    }
  }

  const int jtop = tile - 1;
  __syncthreads();

  // Sort the tile by digit in LDS (keys first, then payloads through the same
  // buffer) and write each digit's run to its global position.
  const int64_t tile_begin = (int64_t)tile * kSortTile;
  const int nvalid =
      kFull ? kSortTile : (int)((P - tile_begin) < kSortTile ? (P - tile_begin) : kSortTile);
  // All slot reads are issued before the stage writes, so their LDS round
  // trips overlap.
  uint32_t pos[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i)
    pos[i] = wcnt[wave][(uint32_t)(key[i] >> shift) & mask] + rank[i];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i)
    if ((kFull || base + i * kWave + lane < P) && pos[i] < (uint32_t)kSortTile)
      stage[pos[i]] = key[i];

  // Decoupled look-back over earlier tiles for this digit (after the LDS sort,
  // which gives predecessors time to publish).
  if (digit_thread) {
    // Consume predecessors nearest first: aggregates are added, a prefix ends
    // the walk.  A predecessor that has not published yet is polled alone,
    // with back-off, so waiting costs one uncached word per poll.
    uint64_t excl = 0ull;
    uint32_t spins = 0u;
    int j = jtop;
    bool done = j < 0;
    while (!done) {
      uint64_t v[kLookWindow];
#pragma unroll
      for (int q = 0; q < kLookWindow; ++q) {
          v[q] = (j - q >= 0) ? __hip_atomic_load(&lb_cur[(size_t)(j - q) * kSortRadix + tid],
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                              : kFlagPrefix;
      }
      int used = 0;
      bool stalled = false;
#pragma unroll
      for (int q = 0; q < kLookWindow; ++q) {
        if (!done && !stalled) {
          const uint64_t f = v[q] & ~kValueMask;
          if (f == 0ull) {
            stalled = true;
          } else {
            excl += v[q] & kValueMask;
            ++used;
            done = f == kFlagPrefix;
          }
        }
      }
      j -= used;
      if (done || j < 0) break;
      if (stalled) {
        uint32_t backoff = 1u;
        uint64_t w;
        while (true) {
          w = __hip_atomic_load(&lb_cur[(size_t)j * kSortRadix + tid], __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
          if ((w & ~kValueMask) != 0ull) break;
          if (++spins > kSpinLimit) break;
          for (uint32_t b = 0; b < backoff; ++b) __builtin_amdgcn_s_sleep(2);
          if (backoff < 16u) backoff <<= 1;
        }
        if (spins > kSpinLimit) {
          atomicOr(status, kStatusInternal);
          break;
        }
        excl += w & kValueMask;
        --j;
        done = (w & ~kValueMask) == kFlagPrefix;
      }
    }
    __hip_atomic_store(&lb_cur[(size_t)tile * kSortRadix + tid], kFlagPrefix | (excl + tcount),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    goff[tid] = dig_off[d * kSortRadix + tid] + (uint32_t)excl - tstart;
  }
  __syncthreads();
  // Each thread visits the same positions j in both write loops; the output
  // index found for the key is kept for the payload.
  // The last pass stores the sorted coordinates themselves (decoded from the
  // keys) in place of the keys: the scans read them as they are.
  const bool last = d == pass->last_pass;
  const Codec<T> cd = codec_of<T>(pass);
  // Stage keys, then their runs' offsets, then the stores: each phase issues
  // all of its LDS reads before any result is used.
  K ks[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int j = tid + r * kSortThreads;
    ks[r] = (kFull || j < nvalid) ? stage[j] : (K)0;
  }
  uint32_t go[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) go[r] = goff[(uint32_t)(ks[r] >> shift) & mask];
  uint32_t outpos[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int j = tid + r * kSortThreads;
    outpos[r] = 0xffffffffu;
    if (kFull || j < nvalid) {
      const uint64_t out = (uint64_t)go[r] + (uint64_t)j;
      if (out < (uint64_t)P) {
        outpos[r] = (uint32_t)out;
        kout[out] = last ? bits_of(cd.decode(ks[r])) : ks[r];
      }
    }
  }
  __syncthreads();
  uint32_t* sid = (uint32_t*)stage;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i)
    if ((kFull || base + i * kWave + lane < P) && pos[i] < (uint32_t)kSortTile) sid[pos[i]] = id[i];
  __syncthreads();
  // The last pass writes the final permutation to its own array, which the
  // scans keep using.
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int j = tid + r * kSortThreads;
    if ((!kFull && j >= nvalid) || outpos[r] == 0xffffffffu) continue;
    const uint32_t out = outpos[r];
    const uint32_t id = sid[j];
    if (last)
      ids_out[out] = id;
    else
      iout[out] = id;
  }
}

template <class T>
__global__ __launch_bounds__(kSortThreads, 4) void k_onesweep(
    int d, const T* __restrict__ x, const T* __restrict__ y, int64_t N,
    int64_t P, void* keys0, void* keys1, uint32_t* idx0, uint32_t* idx1,
    uint32_t* __restrict__ ids_out,
    const uint32_t* __restrict__ dig_off, const PassInfo* __restrict__ pass,
    uint32_t* __restrict__ tile_ctr, uint64_t* lb_cur, uint64_t* lb_next,
    uint32_t* __restrict__ status) {
  __shared__ SweepLds<T> lds;
  __shared__ int s_tile;
  const int tid = threadIdx.x;
  const int run = pass->run[d];
  const int ndig = 1 << pass->bits;
  if (!run) {
    // Nothing moves; still clear the other look-back buffer for the next pass
    // that runs (none after the last: the next sort's first pass starts from
    // the buffer k_clear zeroes, and each pass clears the one after it).
    if (d < pass->last_pass && tid < ndig)
      for (int64_t t = blockIdx.x; t * kSortTile < P; t += gridDim.x)
        lb_next[(size_t)t * kSortRadix + tid] = 0ull;
    return;
  }
  if (tid == 0) s_tile = (int)atomicAdd(&tile_ctr[d], 1u);
  for (int i = tid; i < kSortWaves * kSortRadix; i += kSortThreads) (&lds.wcnt[0][0])[i] = 0;
  if (tid < kSortRadix) lds.thist[tid] = 0u;
  __syncthreads();
  const int tile = s_tile;
  if (tid < ndig) lb_next[(size_t)tile * kSortRadix + tid] = 0ull;
  if ((int64_t)(tile + 1) * kSortTile <= P)
    sweep_tile<T, true>(lds, tile, d, x, y, N, P, keys0, keys1, idx0, idx1, ids_out, dig_off,
                        pass, lb_cur, status);
  else
    sweep_tile<T, false>(lds, tile, d, x, y, N, P, keys0, keys1, idx0, idx1, ids_out, dig_off,
                         pass, lb_cur, status);
}

// Points given in ascending order: the sorted coordinates and identity ids as
// the sort would leave them (the strengths are read in place).  Unsorted input
// raises kStatusUnsorted.
template <class T>
__global__ __launch_bounds__(256) void k_presorted(const T* __restrict__ x, int64_t N,
                                                   T* __restrict__ zs, uint32_t* __restrict__ ids,
                                                   PassInfo* __restrict__ pass,
                                                   uint32_t* __restrict__ status) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool unsorted = false, bad = false;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += stride) {
    const T z = x[p];
    bad |= !isfinite(z);
    if (p > 0) unsorted |= !(z >= x[p - 1]);
    zs[p] = z;
    ids[p] = (uint32_t)p;
  }
  if (unsorted) atomicOr(status, kStatusUnsorted);
  if (bad) atomicOr(status, kStatusNonFinite);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    pass->final_buf = 0;
    pass->last_pass = -1;
  }
}

// The sorted state left by the last sort: merged index and coordinate of every
// sorted position (either output may be null).
template <class T>
__global__ __launch_bounds__(256) void k_copy_sorted(const void* keys0, const void* keys1,
                                                     const PassInfo* __restrict__ pass,
                                                     const uint32_t* __restrict__ ids, int64_t P,
                                                     uint32_t* __restrict__ perm,
                                                     T* __restrict__ z) {
  const KeyView<T> keys = key_view<T>(keys0, keys1, pass);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += stride) {
    if (perm) perm[p] = ids[p];
    if (z) z[p] = keys(p);
  }
}

}  // namespace

template <class T>
hipError_t presorted_points(const Workspace& w, const T* x, const T* alpha, int64_t N,
                            hipStream_t s) {
  (void)alpha;
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, s, w.status, (size_t)64);
  int64_t blocks = (N + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_presorted<T>, dim3((unsigned)blocks), dim3(256), 0, s, x, N, (T*)w.keys[0],
                     w.ids, w.pass, w.status);
  return hipGetLastError();
}

template <class T>
hipError_t copy_sorted(const Workspace& w, int64_t P, uint32_t* perm, T* z, hipStream_t s) {
  int64_t blocks = (P + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy_sorted<T>, dim3((unsigned)blocks), dim3(256), 0, s, w.keys[0], w.keys[1],
                     w.pass, w.ids, P, perm, z);
  return hipGetLastError();
}
template hipError_t copy_sorted<double>(const Workspace&, int64_t, uint32_t*, double*, hipStream_t);
template hipError_t copy_sorted<float>(const Workspace&, int64_t, uint32_t*, float*, hipStream_t);

template hipError_t presorted_points<double>(const Workspace&, const double*, const double*,
                                             int64_t, hipStream_t);
template hipError_t presorted_points<float>(const Workspace&, const float*, const float*, int64_t,
                                            hipStream_t);

template <class T>
hipError_t sort_points(const Workspace& w, const T* x, int64_t M, const T* y, int64_t N,
                       const SortRes& res, hipStream_t s, Timeline* tl) {
  constexpr int D = KeyOf<T>::kDigits;
  const int64_t P = M + N;
  tl->mark(s);
  const size_t words = w.zero_bytes / 4;
  hipLaunchKernelGGL(k_clear, dim3((unsigned)((words + 255) / 256 < 4096 ? (words + 255) / 256 : 4096)),
                     dim3(256), 0, s, w.status, words);
  int64_t hb = (P + 256 * 16 - 1) / (256 * 16);
  if (hb > kHistBlocks) hb = kHistBlocks;
  if (hb < 1) hb = 1;
  if (sizeof(T) == 8)
    // Few large blocks: each block ends with atomics on the same three words.
    hipLaunchKernelGGL(k_range<T>, dim3((unsigned)(hb < 256 ? hb : 256)), dim3(1024), 0, s, x, y,
                       N, P, w.range, w.status);
  hipLaunchKernelGGL(k_histogram<T>, dim3((unsigned)hb), dim3(256), 0, s, x, y, N, P, w.hist,
                     w.status, w.range, res);
  hipLaunchKernelGGL(k_plan<T>, dim3(1), dim3(512), 0, s, w.hist, P, w.range, res, w.dig_off,
                     w.pass);
  tl->mark(s);
  for (int d = 0; d < D; ++d) {
    hipLaunchKernelGGL(k_onesweep<T>, dim3((unsigned)w.sort_tiles), dim3(kSortThreads), 0, s, d, x,
                       y, N, P, w.keys[0], w.keys[1], w.idx[0], w.idx[1], w.ids,
                       w.dig_off, w.pass,
                       w.tile_ctr, w.lookback[d & 1], w.lookback[(d + 1) & 1], w.status);
    tl->mark(s);
  }
  return hipGetLastError();
}

template hipError_t sort_points<double>(const Workspace&, const double*, int64_t, const double*,
                                        int64_t, const SortRes&, hipStream_t, Timeline*);
template hipError_t sort_points<float>(const Workspace&, const float*, int64_t, const float*,
                                       int64_t, const SortRes&, hipStream_t, Timeline*);

}  // namespace fgt
