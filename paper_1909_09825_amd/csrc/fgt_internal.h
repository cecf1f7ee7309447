// Internal definitions shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fgt.h"

namespace fgt {

// ---------------------------------------------------------------------------
// SOE table as shipped (delta = 1) and as a kernel argument (scaled to delta).
// ---------------------------------------------------------------------------
struct SoeTable {
  int n_modes;
  double tau0_re[FGT_MAX_MODES], tau0_im[FGT_MAX_MODES];
  double om_re[FGT_MAX_MODES], om_im[FGT_MAX_MODES];
  double err_bound, deriv_err_bound, sum_abs_omega;
};

// Highest Taylor degree of the mode exponential and highest power moment.
constexpr int kTaylorMax = 12;
constexpr int kMomentMax = 20;

// Passed by value to the scan kernels: tau_k = tau0_k / sqrt(delta), omega_k,
// |tau_k|, max_k |tau_k|, and the Taylor thresholds of the plan's precision:
// degree D is enough for exp(-w) when |w| <= taylor_thr[D], i.e.
// taylor_thr[D]^{D+1} / (D+1)! equals the unit roundoff.
// Sort resolution.  With IEEE order keys, coordinates closer than key_width
// may be left unordered; with the FP64 grid code (Codec<double>) the points
// may also move by up to code_tol, and both take half of the allowance:
// key_width_q, code_tol.
struct SortRes {
  double key_width;
  double key_width_q;
  double code_tol;
};

struct Modes {
  int n;
  double tau_re[FGT_MAX_MODES], tau_im[FGT_MAX_MODES];
  double om_re[FGT_MAX_MODES], om_im[FGT_MAX_MODES];
  double tau_abs[FGT_MAX_MODES];
  double tau_abs_max;
  double taylor_thr[kTaylorMax + 1];
  double key_width;   // sort resolution in coordinate units (see fgt_plan)
  SortRes sort;
  // Largest gap whose exponential the degree-kTaylorMax polynomial serves:
  // taylor_thr[kTaylorMax] / |tau_k|.
  double dz_lim[FGT_MAX_MODES];
  // Taylor coefficients of exp(-tau_k x) in x: (-tau_k)^m / m!.
  double coef_re[FGT_MAX_MODES][kTaylorMax + 1];
  double coef_im[FGT_MAX_MODES][kTaylorMax + 1];
  // Weights of the derivative field: d/dx exp(-tau |x|) = -tau sign(x) exp(-tau |x|),
  // so S'(x) = Re sum_k dom_k sign(x) exp(-tau_k |x|) with dom_k = -tau_k omega_k.
  double dom_re[FGT_MAX_MODES], dom_im[FGT_MAX_MODES];
};

// What the final scan kernel writes.  Sorted point p carries its merged index
// id_p; it is an output point when o = id_p - t_lo < t_n, and then
//   val[o] = sum_k Re(omega_k (h+ + h-))                      (the transform, (4.1))
//   der[o] = scale[o] * sum_k Re(dom_k (h+ - h-))             (its x-derivative)
// (scale null: factor 1).  The unsigned compare keeps every write in bounds.
template <class T>
struct ScanOut {
  T* val;
  T* der;
  const T* scale;
  uint32_t t_lo, t_n;
};
constexpr int kOutVal = 1;
constexpr int kOutDer = 2;

// ---------------------------------------------------------------------------
// Tunables.
// ---------------------------------------------------------------------------
constexpr int kWave = 64;

// LSD radix sort: 8-bit digits, one-sweep passes with decoupled look-back.
constexpr int kSortThreads = 512;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // 8192 keys per tile
constexpr int kRadix = 256;
// Digits of the single-transform sort: 8 or 9 bits, chosen per call on the
// device (the batched bucket sort keeps 8-bit digits); tables are sized for 9.
constexpr int kSortBits = 9;
constexpr int kSortRadix = 1 << kSortBits;
constexpr int kHistBlocks = 2048;

// Scan: each thread owns a run of kScanChunk consecutive sorted points.
constexpr int kScanThreads = 256;
constexpr int kScanWaves = kScanThreads / kWave;
constexpr int kScanChunk = 8;
constexpr int kScanTile = kScanThreads * kScanChunk;   // 2048 points per tile (adjoint)
// Forward scan: a tile is one wave, kScanChunk consecutive points per lane.
constexpr int kWTile = kWave * kScanChunk;             // 512 points per tile
constexpr int kCarryThreads = 1024;
// Per tile and mode the reduce kernel stores A, F, G and the two factors
// exp(-tau hf), exp(-tau hg) that move the tile carries to its centre.
constexpr int kAggStride = 10;
// Tiles whose moment count is at most this take the fast final kernel.
constexpr int kFastMoments = 12;


template <class T> struct KeyOf;
template <> struct KeyOf<double> { using type = uint64_t; static constexpr int kDigits = 8; };
template <> struct KeyOf<float> { using type = uint32_t; static constexpr int kDigits = 4; };

// Order-preserving map from a float to an unsigned key: negative values get
// all bits flipped, non-negative ones the sign bit set; -0 is mapped to +0 so
// that equal coordinates get equal keys.  (Host and device: the key code below
// is also checked on the CPU.)
__host__ __device__ __forceinline__ uint64_t to_key(double z) {
  uint64_t b = __builtin_bit_cast(uint64_t, z);
  if (b == 0x8000000000000000ull) b = 0;
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ uint32_t to_key(float z) {
  uint32_t b = __builtin_bit_cast(uint32_t, z);
  if (b == 0x80000000u) b = 0;
  return (b >> 31) ? ~b : (b | 0x80000000u);
}
__host__ __device__ __forceinline__ double from_key(uint64_t k) {
  const uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __builtin_bit_cast(double, b);
}
__host__ __device__ __forceinline__ float from_key(uint32_t k) {
  const uint32_t b = (k >> 31) ? (k & 0x7fffffffu) : ~k;
  return __builtin_bit_cast(float, b);
}

__host__ __device__ __forceinline__ uint64_t bits_of(double z) {
  return __builtin_bit_cast(uint64_t, z);
}
__host__ __device__ __forceinline__ uint32_t bits_of(float z) {
  return __builtin_bit_cast(uint32_t, z);
}

// Sort keys as the radix passes see them.  FP32 coordinates keep their IEEE
// order keys.  FP64 coordinates are, where that loses nothing that matters,
// coded as fixed-point offsets on a power-of-two grid g fitted to the range
// [lo, hi] of the call's points (keys below 2^63): the key bits are spent on
// the occupied interval, and more low digits fall below the sort resolution
// and are skipped.  Coordinates on the grid (those with ulp(z) >= g, or all of
// them when the range sits far from 0) decode exactly; smaller ones are
// truncated by less than g, and the code is used only when such a shift is
// within the plan's tolerance (else IEEE keys).
template <class T> struct Codec;
template <> struct Codec<double> {
  double L;        // offset subtracted before scaling (exact by Sterbenz), or 0
  double g, inv_g; // grid step 2^e and its inverse
  int64_t F;       // grid index of the range's aligned start when L = 0
  int32_t quant;   // 0: IEEE order keys
  __host__ __device__ __forceinline__ uint64_t encode(double z) const {
    if (!quant) return to_key(z);
    double t = (z - L) * inv_g;                 // exact for grid points, below 2^63
    const double t0 = (double)F;                // exact
    const double top = 9223372036854773760.0;   // 2^63 - 2048: the int64 conversion stays defined
    t = t > t0 ? t : t0;                        // (NaN lands here too)
    t = t < top ? t : top;
    return (uint64_t)(int64_t)t - (uint64_t)F;
  }
  __host__ __device__ __forceinline__ double decode(uint64_t q) const {
    if (!quant) return from_key(q);
    return fma((double)(int64_t)(q + (uint64_t)F), g, L);
  }
};
template <> struct Codec<float> {
  __host__ __device__ __forceinline__ uint32_t encode(float z) const { return to_key(z); }
  __host__ __device__ __forceinline__ float decode(uint32_t k) const { return from_key(k); }
};

// Exponent of the largest power of two that divides z (finite, non-zero): the
// value of its lowest set significand bit.  Branch-free: a normal number's
// implicit bit is bit 52 and its scale 2^(e-1075); a subnormal's scale is
// 2^-1074 and its significand is below 2^52, so setting bit 52 changes no
// trailing zero count that matters.
__host__ __device__ __forceinline__ int granularity_exp(double z) {
  const uint64_t b = __builtin_bit_cast(uint64_t, z) & 0x7fffffffffffffffull;
  const int e = (int)(b >> 52);
  return (e > 1 ? e : 1) - 1075 + (int)__builtin_ctzll(b | (1ull << 52));
}

// Code for points whose smallest and largest IEEE order keys are kmin, kmax.
// With span = hi - lo < 2^E the range starts at lo_a = floor(lo / 2^E) 2^E, so
// every point lies in [lo_a, lo_a + 2^(E+1)).  If |lo_a| >= 2^(E+2) all points
// share lo_a's sign and lie within a factor 2 of it: z - lo_a is exact and a
// multiple of g = 2^(E-62), and the keys (z - lo_a) / g are below 2^63.
// Otherwise the keys are z / g - lo_a / g (exact power-of-two scaling) with g
// the smallest power of two that keeps |z| / g and the keys below 2^63.  A
// point is on that grid when it is a multiple of g; `gran` is the exponent of
// the largest power of two that every point is a multiple of (see
// granularity_exp; very large when unknown points are all zero).  If some
// point is finer than g it moves by less than g, which must not exceed
// code_tol.  Degenerate ranges (non-finite, all equal, extreme exponents) keep
// IEEE keys.
__host__ __device__ __forceinline__ Codec<double> make_codec(uint64_t kmin, uint64_t kmax,
                                                             int gran, double code_tol) {
  Codec<double> c{0.0, 0.0, 0.0, 0, 0};
  const double lo = from_key(kmin), hi = from_key(kmax);
  if (!(isfinite(lo) && isfinite(hi) && hi > lo)) return c;
  const double span = hi - lo;
  if (!isfinite(span)) return c;
  int E = 0;
  (void)frexp(span, &E);                        // span < 2^E
  if (E > 1000 || E < -900) return c;
  const double pE = ldexp(1.0, E);
  double lo_a = floor(lo / pE) * pE;
  if (lo_a > lo) lo_a -= pE;
  int eg = E - 62;
  if (fabs(lo_a) >= 4.0 * pE) {
    c.L = lo_a;
    c.F = 0;
  } else {
    const double m = fabs(lo_a) > fabs(hi) ? fabs(lo_a) : fabs(hi);
    int em = 0;
    (void)frexp(m, &em);                        // |z| <= m < 2^em
    if (em - 63 > eg) eg = em - 63;
    if (gran < eg && !(ldexp(1.0, eg) <= code_tol)) return c;
    c.L = 0.0;
    c.F = (int64_t)(lo_a * ldexp(1.0, -eg));
  }
  c.g = ldexp(1.0, eg);
  c.inv_g = ldexp(1.0, -eg);
  c.quant = 1;
  return c;
}

struct PassInfo {
  int32_t run[8];     // 1 if radix pass d moves data
  int32_t src[8];     // 0/1: key buffer it reads, 2: the raw coordinates
  int32_t final_buf;  // buffer that holds the sorted coordinates at the end
  int32_t last_pass;  // the last pass that runs; it also writes the coordinates and ids
  int32_t skipped_low;  // low key bits left unsorted (below the plan's key resolution)
  int32_t shift[8];     // lowest bit of pass d's digit
  int32_t bits;         // digit width of this sort, 8 or 9
  int32_t code_quant;   // FP64 key code of this sort's keys (Codec<double>)
  int64_t code_F;
  double code_L, code_g, code_inv_g;
};

template <class T>
__device__ __forceinline__ Codec<T> codec_of(const PassInfo* pass) {
  if constexpr (sizeof(T) == 8) {
    return Codec<double>{pass->code_L, pass->code_g, pass->code_inv_g, pass->code_F,
                         pass->code_quant};
  } else {
    (void)pass;
    return Codec<float>{};
  }
}

// The sorted coordinates left by the last sort (its last pass stores them in
// place of the keys).
template <class T>
struct KeyView {
  const T* z;
  __device__ __forceinline__ T operator()(int64_t p) const { return z[p]; }
};
template <class T>
__device__ __forceinline__ KeyView<T> key_view(const void* keys0, const void* keys1,
                                               const PassInfo* pass) {
  return KeyView<T>{(const T*)(pass->final_buf ? keys1 : keys0)};
}

// Merged index given to padding past the last point (never an output).
constexpr uint32_t kNoSlot = 0xffffffffu;

// Bits of the device status word.
constexpr uint32_t kStatusNonFinite = 1u;
constexpr uint32_t kStatusInternal = 2u;
constexpr uint32_t kStatusUnsorted = 4u;

// ---------------------------------------------------------------------------
// Workspace layout (all offsets 256-byte aligned).
// ---------------------------------------------------------------------------

struct Workspace {
  void* keys[2];         // [P] each: radix keys; the last pass leaves the sorted coordinates
  uint32_t* idx[2];
  void* b;               // [P] strength of each sorted point (alpha_j for a source, 0 for a target)
  uint32_t* ids;         // [P] merged index of each sorted point: j < N source j, else target j - N
  void* bt;              // [P] strengths of the transposed transform (g_i at targets, 0 at
                         //     sources); shares the permutation buffers, which are dead after the sort
  double* tile_part;     // [scan_tiles] per-tile parts of the delta-gradient sum
  uint32_t* status;      // [1] at offset 0, zeroed per call
  unsigned long long* range;   // [3] ~(smallest key), largest key (IEEE order), and (FP64)
                               // 2048 - the finest granularity exponent of the points; zeroed per call
  uint32_t* hist;        // [digits][256], zeroed per call
  uint32_t* tile_ctr;    // [8], zeroed per call
  uint64_t* lookback[2]; // [sort_tiles][256]; [0] zeroed per call, each pass clears the other
  uint32_t* dig_off;     // [digits][256]
  PassInfo* pass;
  void* agg;             // [tiles][scans][kAggStride] scalars (complex A, F, G, eF, eG): the
                         // forward's wave_tiles x modes, or the adjoint's scan_tiles x 2 modes
  int32_t* tile_k;       // [tiles] moments used for the tile, -1 if it is too wide
  void* carry;           // [tiles][scans][4] scalars: CF, CB (complex)
  void* chunk_agg;       // [chunks][modes][6]: composed (A, F, G) of 64 consecutive tiles
  void* chunk_carry;     // [chunks][modes][4]: CF, CB entering each chunk
  void* small_part;      // [modes][P] per-mode sums of the one-launch path (P <= kSmallMax), else null
  size_t zero_bytes;     // bytes from `status` that the first kernel clears
  int64_t sort_tiles, scan_tiles, wave_tiles;   // radix tiles, adjoint scan tiles, forward scan tiles
  size_t total;
};

// Transforms with P = M + N up to this run as one block per mode (fgt_small.hip).
constexpr int kSmallMax = 4096;

// Phase boundaries for benchmark timing: mark() records the next event, if any.
constexpr int kMaxPhases = 12;   // setup, 8 radix passes, tile reduce, carry, tile final
struct Timeline {
  hipEvent_t* ev = nullptr;
  int n = 0, cap = 0;   // n: marks made (recorded while n < cap)
  void mark(hipStream_t s) {
    if (!ev) return;
    if (n < cap) (void)hipEventRecord(ev[n], s);
    ++n;
  }
};

// Smallest shipped table with E_n <= 10^-digits (null if none).
const SoeTable* choose_table(int digits);
// Largest digits served for an element type.
int max_digits(int dtype);
// Scale a table to delta and fill the kernel constants for the element type.
void make_modes(const SoeTable* tab, double delta, int dtype, Modes* m);

// Layout for P points, element size `esz` (8 or 4), n_modes modes.  With
// base == nullptr only sizes are computed.
Workspace layout(void* base, int64_t P, int esz, int n_modes);

// Kernel launch sequences (defined in the .hip files).
// res: coordinate differences below the resolution may be left unordered;
// zero widths sort every digit, a zero code_tol keeps IEEE keys wherever the
// grid code would move a point.
template <class T>
hipError_t sort_points(const Workspace& w, const T* x, int64_t M, const T* y, int64_t N,
                       const SortRes& res, hipStream_t s, Timeline* tl);
// Scan over the sorted coordinates; writes what `out` asks for.  The strengths
// in sorted order are `b` ([P]) when `src` is null; otherwise the tile reduce
// gathers them, b_p = src[id_p] for id_p < n_src and 0 else, and stores them
// to w.b for the kernels after it.
template <class T>
hipError_t scan_points(const Workspace& w, const Modes& m, int64_t P, const T* b, const T* src,
                       uint32_t n_src, const ScanOut<T>& out, hipStream_t s, Timeline* tl);
// b[p] = wts[id_p - lo] if that index is below n, else 0.
template <class T>
hipError_t gather_strengths(const Workspace& w, int64_t P, uint32_t lo, uint32_t n, const T* wts,
                            T* b, hipStream_t s);
// Gradients of L = sum_i g_i u_i from the sorted state of the last forward
// call (keys, ids, and the forward strengths b); any output may be null.
template <class T>
hipError_t adjoint_points(const Workspace& w, const Modes& md, int64_t M, int64_t N, const T* g,
                          T* dx, T* dalpha, T* dy, T* ddelta, double delta, hipStream_t s);
// Copy the sorted state (merged ids, sorted coordinates) to caller arrays (either may be null).
template <class T>
hipError_t copy_sorted(const Workspace& w, int64_t P, uint32_t* perm, T* z, hipStream_t s);
template <class T>
hipError_t fill_zero(T* u, int64_t n, hipStream_t s);
// Points given in ascending order: coordinates and identity ids written as the sort
// would leave them (the scan then reads alpha in place); order and finiteness
// checked.
template <class T>
hipError_t presorted_points(const Workspace& w, const T* x, const T* alpha, int64_t N,
                            hipStream_t s);

// ---------------------------------------------------------------------------
// Batched transforms (B independent transforms in CSR layout, R strength
// columns).  Coordinates of transform b are scaled by s_b = 1/sqrt(delta_b),
// so one table at delta = 1 serves every transform.
// ---------------------------------------------------------------------------
// Sort: each transform's merged points [sources; targets] are split by the top
// bits of a quantised key into buckets of about kBucketTarget points (stable
// counting per chunk of kBChunk points), then every bucket is radix-sorted in
// LDS (kBucketMax points at most; larger buckets take a slower block-global path).
constexpr int kBChunk = 4096;
constexpr int kBucketMax = 4096;
constexpr int kBSortThreads = 512;
constexpr int kBSortItems = kBucketMax / kBSortThreads;   // 8
constexpr int kMaxBucketLog2 = 12;
// Scan: a wave holds 4 chunks x 16 columns, a lane runs consecutive points
// of one column.
constexpr int kBCols = 16;
constexpr int kBThreads = 256;
// Points per lane and column: 8 or 16 (chosen per batch by the autotuner);
// a tile holds (kBThreads / kBCols) chunks.
constexpr int kBTileMin = (kBThreads / kBCols) * 8;   // 128
// Bit of a sorted id that marks the first point of a transform.
constexpr uint32_t kSegStart = 0x80000000u;

struct SegInfo {
  int64_t x_off, y_off;   // first target row, first source row
  int64_t M, N;           // targets, sources
  int64_t base;           // first sorted position of the transform
  int64_t chunk0;         // first chunk of the transform
  int64_t bucket0;        // first bucket of the transform
  int64_t cnt0;           // first entry of its [bucket][chunk] count table
  double scale;           // 1 / sqrt(delta_b)
  int32_t n_chunks;
  int32_t nb_log2;        // log2 of its bucket count
};
struct ChunkInfo {
  int32_t seg;
  int32_t pad;
  int64_t start;          // first merged index of the chunk inside its transform
};
struct BucketInfo {
  int32_t seg;
  int32_t idx;
};

struct BatchWork {
  uint32_t* status;       // [64] at offset 0
  double* lo;             // [B] smallest scaled coordinate per transform
  double* hi;             // [B] largest
  uint32_t* counts;       // [sum n_chunks * nb] bucket-major per transform
  uint32_t* offs;         // [same] exclusive offsets
  uint32_t* bstart;       // [sum nb] bucket start inside its transform
  uint32_t* bsize;        // [sum nb]
  uint32_t* ids_tmp;      // [P] merged indices after the bucket split
  double* z_tmp;          // [P] their coordinates (unscaled), beside them
  uint64_t* qbuf[2];      // [P] keys of the block-global path
  uint32_t* ibuf[2];      // [P]
  double* zs;             // [P] sorted coordinates
  uint32_t* ids;          // [P] sorted codes: source row, or SN + target row; kSegStart flag
  double* tile_a;         // [tiles][modes][2]
  double* tile_fg;        // [tiles][modes][R][4]
  double* chunk_agg;      // [chunks][modes * R][6]
  double* chunk_carry;    // [chunks][modes * R][4]
  double* carry;          // [tiles][modes * R][4]
  size_t total;
};

// Device tables of a batch plan for one bucket size.
struct BatchTables {
  const SegInfo* seg;
  const ChunkInfo* chunks;
  const BucketInfo* buckets;
  const int64_t* ne_base;
  const double* ne_scale;
  int64_t n_buckets;
  int max_nb_log2;
};

struct BatchDims {
  int64_t B, P, SN, SM, n_chunks, n_buckets, n_counts, tiles;
  int64_t K;              // transforms with at least one point
  int R, n_modes;
};

BatchWork batch_layout(void* base, const BatchDims& d);

// The whole batch: sort, then the scan with `chunk` (8 or 16) points per lane.
// d sizes the workspace (maxima over the tunable choices); t holds the tables
// of the chosen bucket size.
hipError_t batch_eval_launch(const BatchDims& d, const BatchTables& t, const Modes& md,
                             double s_allow, int chunk, const double* x, const double* y,
                             const double* alpha, double* u, const BatchWork& w, hipStream_t s);

// The sorted codes (kSegStart cleared) and coordinates a batch left in w.
hipError_t batch_sorted_copy(const BatchDims& d, const BatchWork& w, uint32_t* codes, double* z,
                             hipStream_t s);

}  // namespace fgt
