// The SOE recurrences of Section 4 as parallel affine scans on gfx950.
//
// After the sort, point p of the merged sequence has coordinate z_p,
// strength b_p (alpha_j for source j, 0 for a target) and its merged index,
// which names the output it feeds.  For mode k (tau = tau0_k / sqrt(delta)) let
//     e_p = exp(-tau (z_p - z_{p-1})),   |e_p| <= 1 since z is sorted.
// The forward recurrence (4.5) over the merged sequence is
//     h+_p = e_p h+_{p-1} + b_p          (inclusive: sources at z_p count, (4.4))
// and the backward recurrence (4.6), exclusive of the point itself, is
//     h-_{p-1} = e_p (h-_p + b_p).
// One factor e_p serves both.  At a target u_p = sum_k Re(omega_k (h+_p + h-_p)), (4.1).
//
// A segment [s, e) of the sequence acts on the two recurrences as
//     h+_{e-1} = A h+_{s-1} + F,          h-_{s-1} = A h-_{e-1} + G,
//     A = prod_{p in seg} e_p = exp(-tau (z_{e-1} - z_{s-1})),
//     F = sum_{q in seg} b_q exp(-tau (z_{e-1} - z_q)),   G = sum_{q in seg} b_q exp(-tau (z_q - z_{s-1})),
// and segments compose associatively:  (A1,F1,G1).(A2,F2,G2) = (A1 A2, A2 F1 + F2, G1 + A1 G2).
//
// Reduce-then-scan over tiles of kWTile points.  A tile is one wave: lane l
// holds the kScanChunk consecutive points [t0 + l C, t0 + (l + 1) C), read
// straight into registers, so the kernels need no LDS and no barrier (a block
// of 256 threads runs 4 independent tiles):
//   k_wreduce     the tile's (A, F, G) for every mode.  When the tile is short on
//                 the decay scale (|tau| times its half-width small) the sums come
//                 from mode-independent power moments of the strengths about the
//                 tile centre c:  sum_q b_q exp(+-tau (z_q - c)) =
//                 sum_m (+-tau)^m mu_m / m!,  mu_m = sum_q b_q (z_q - c)^m;
//                 otherwise from the recurrences themselves.
//   carries       per mode: exclusive prefix of F and suffix of G over tiles.
//   k_wfinal_fast tiles short on the decay scale: the value entering each lane's
//                 chunk from the moments of the tile's other chunks, both sweeps,
//                 the sum over modes, scatter to the outputs.
//   k_wfinal      the other tiles: lane maps, wave scans of both recurrences.
// The number of moments is a compile-time constant in every loop (the tile's
// count rounded up to one of a few values), so no loop runs masked slots.
#include "fgt_device.h"

namespace fgt {
namespace {

// Moment counts the kernels are compiled for; a tile takes the smallest that
// is not below its own count.
constexpr int kKSteps[] = {2, 4, 6, 8, 12, 16, 20};
static_assert(kKSteps[4] == kFastMoments, "the fast final kernel serves counts up to kFastMoments");

__device__ __forceinline__ int k_class(int K) {
  int c = 0;
#pragma unroll
  for (int i = 6; i >= 0; --i)
    if (K <= kKSteps[i]) c = i;
  return c;
}

// Moments needed for a tile whose points lie within r / max|tau| of its
// centre: the series tail r^{K+1}/(K+1)! e^r must be below the unit roundoff;
// -1 when kMomentMax terms are not enough.  For r <= 1, e^r <= 1 + r + r^2
// stands in for the exponential (a bound, so the count is never too small).
template <class T>
__device__ __forceinline__ int moment_count(T r) {
  int K = 0;
  const T er = r <= T(1) ? T(1) + r + r * r : exp_t(r);
  T t = r;
  while (t * er > T(Prec<T>::kUnit) && K < kMomentMax) {
    ++K;
    t *= r / T(K + 1);
  }
  return t * er > T(Prec<T>::kUnit) ? -1 : K;
}

// A lane's chunk of the tile: coordinates, strengths (and merged ids),
// loaded with 16-byte loads when the arrays allow it.  The loads are cached:
// the lanes of a wave read 64 bytes apart, so each line serves several of
// the loads (with the nontemporal hint the kernels ran 15-30% slower).
// Points past the end read as z = 0, b = 0, id = kNoSlot.
template <class T>
__device__ __forceinline__ void load_chunk(const T* __restrict__ z, const T* __restrict__ b,
                                           int64_t base, int64_t P, bool vec, T* zc, T* bc) {
  constexpr int C = kScanChunk;
  if (vec && base + C <= P) {
    typedef T V __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int L = 16 / sizeof(T);
    const V* pz = reinterpret_cast<const V*>(z + base);
    const V* pb = reinterpret_cast<const V*>(b + base);
#pragma unroll
    for (int q = 0; q < C / L; ++q) {
      const V vz = pz[q];
      const V vb = pb[q];
#pragma unroll
      for (int i = 0; i < L; ++i) {
        zc[q * L + i] = vz[i];
        bc[q * L + i] = vb[i];
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int64_t p = base + j;
      zc[j] = p < P ? z[p] : T(0);
      bc[j] = p < P ? b[p] : T(0);
    }
  }
}

__device__ __forceinline__ void load_ids(const uint32_t* __restrict__ ids, int64_t base, int64_t P,
                                         bool vec, uint32_t* ic) {
  constexpr int C = kScanChunk;
  if (vec && base + C <= P) {
    typedef uint32_t V __attribute__((ext_vector_type(4)));
    const V* pi = reinterpret_cast<const V*>(ids + base);
#pragma unroll
    for (int q = 0; q < C / 4; ++q) {
      const V v = pi[q];
#pragma unroll
      for (int i = 0; i < 4; ++i) ic[q * 4 + i] = v[i];
    }
  } else {
#pragma unroll
    for (int j = 0; j < C; ++j) ic[j] = base + j < P ? ids[base + j] : kNoSlot;
  }
}

// The tile reduce's gather of the strengths in sorted order: the lane's
// coordinates and merged ids, then b_j = src[id_j] for a source (id_j < n) and
// 0 for a target, stored to b for the kernels after the reduce.  The random
// reads overlap the other waves' streams, which a separate gather pass (or
// the last radix pass) would leave idle.
template <class T>
__device__ __forceinline__ void load_gather(const T* __restrict__ z,
                                            const uint32_t* __restrict__ ids,
                                            const T* __restrict__ src, uint32_t n,
                                            T* __restrict__ b, int64_t base, int64_t P, bool vec,
                                            T* zc, T* bc) {
  constexpr int C = kScanChunk;
  uint32_t ic[C];
  load_ids(ids, base, P, vec, ic);   // kNoSlot past the end
  const bool full = vec && base + C <= P;
  typedef T V __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int L = 16 / sizeof(T);
  if (full) {
    const V* pz = reinterpret_cast<const V*>(z + base);
#pragma unroll
    for (int q = 0; q < C / L; ++q) {
      const V vz = pz[q];
#pragma unroll
      for (int i = 0; i < L; ++i) zc[q * L + i] = vz[i];
    }
  } else {
#pragma unroll
    for (int j = 0; j < C; ++j) zc[j] = base + j < P ? z[base + j] : T(0);
  }
#pragma unroll
  for (int j = 0; j < C; ++j) bc[j] = ic[j] < n ? src[ic[j]] : T(0);
  if (full) {
    V* pb = reinterpret_cast<V*>(b + base);
#pragma unroll
    for (int q = 0; q < C / L; ++q) {
      V v;
#pragma unroll
      for (int i = 0; i < L; ++i) v[i] = bc[q * L + i];
      pb[q] = v;
    }
  } else {
#pragma unroll
    for (int j = 0; j < C; ++j)
      if (base + j < P) b[base + j] = bc[j];
  }
}

// Geometry of a wave's tile.  zs: the point before the lane's chunk (the
// tile's previous point for lane 0); ze: the lane's last point (the tile's
// last point for a lane past the end); dz, sc: gaps and offsets from the tile
// centre c (0 for points past the end).
template <class T>
struct TileGeo {
  T zprev, zlast, c, hf, hg, span, zs, ze, dzmax;
  int n;   // points in the tile
};

template <class T>
__device__ __forceinline__ TileGeo<T> tile_geometry(const T* __restrict__ z, int64_t t0, int64_t P,
                                                    int lane, const T* zc, T* dz, T* sc) {
  constexpr int C = kScanChunk;
  TileGeo<T> g;
  g.n = (int)((P - t0) < kWTile ? (P - t0) : kWTile);
  const T zfirst = z[t0];
  g.zprev = t0 > 0 ? z[t0 - 1] : zfirst;
  const int e0 = lane * C;
  // last valid point of the lane (or the point before its chunk when it has none)
  T zl_own = zc[0];
#pragma unroll
  for (int j = 1; j < C; ++j)
    if (e0 + j < g.n) zl_own = zc[j];
  g.zlast = __shfl(zl_own, (g.n - 1) / C, kWave);
  if (e0 >= g.n) zl_own = g.zlast;   // lanes past the end: empty chunks at the last point
  const T up = shfl_up(zl_own, 1);
  g.zs = lane == 0 ? g.zprev : up;
  g.ze = zl_own;
  g.c = g.zprev + (g.zlast - g.zprev) * T(0.5);
  g.hf = g.zlast - g.c;
  g.hg = g.c - g.zprev;
  g.span = g.zlast - g.zprev;
  T zl = g.zs;
  T dm = T(0);
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const bool valid = e0 + j < g.n;
    dz[j] = valid ? zc[j] - zl : T(0);
    sc[j] = valid ? zc[j] - g.c : T(0);
    zl = valid ? zc[j] : zl;
    dm = dz[j] > dm ? dz[j] : dm;
  }
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const T other = shfl_xor(dm, o);
    dm = other > dm ? other : dm;
  }
  g.dzmax = dm;
  return g;
}

// exp(-tau dz_j) for the chunk's gaps: the Taylor polynomial of the wave's
// degree (the smallest whose truncation at the wave's largest gap is below the
// unit roundoff), the library functions for gaps beyond its range.
template <class T>
__device__ __forceinline__ void mode_exps(const Modes& md, int k, const T* dz, T dzmax,
                                          C<T>* ex) {
  const double rr = md.tau_abs[k] * (double)dzmax;
  int D = kTaylorMax;
#pragma unroll
  for (int d = kTaylorMax; d >= 1; --d)
    if (rr <= md.taylor_thr[d]) D = d;
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) ex[j] = {T(0), T(0)};
#pragma unroll
  for (int m = kTaylorMax; m >= 0; --m) {
    if (m <= D) {
      const T c_re = T(md.coef_re[k][m]), c_im = T(md.coef_im[k][m]);
#pragma unroll
      for (int j = 0; j < kScanChunk; ++j) {
        ex[j].re = fma(ex[j].re, dz[j], c_re);
        ex[j].im = fma(ex[j].im, dz[j], c_im);
      }
    }
  }
  const T dz_lim = T(md.dz_lim[k]);
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j)
    if (dz[j] > dz_lim) ex[j] = exp_neg_general<T>(T(md.tau_re[k]), T(md.tau_im[k]), dz[j]);
}

// ---------------------------------------------------------------------------
// k_wreduce: (A, F, G, e^{-tau hf}, e^{-tau hg}) of every tile and mode.
// ---------------------------------------------------------------------------
template <class T, int NM, int KK>
__device__ __forceinline__ void reduce_moments(const Modes& md, const T* bc, const T* sc,
                                               const TileGeo<T>& g, int lane,
                                               T* __restrict__ out) {
  T mu[KK + 1];
#pragma unroll
  for (int m = 0; m <= KK; ++m) mu[m] = T(0);
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    T pw = bc[j];
    mu[0] += pw;
#pragma unroll
    for (int m = 1; m <= KK; ++m) {
      pw *= sc[j];
      mu[m] += pw;
    }
  }
  // Wave totals (the same, order-fixed sum in every lane).
#pragma unroll
  for (int m = 0; m <= KK; ++m) mu[m] = wave_total(mu[m]);
  if (lane < NM) {
    const int k = lane;
    const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
    C<T> fs = {mu[KK] * T(kInvFact.v[KK]), T(0)};
    C<T> gs = fs;
#pragma unroll
    for (int m = KK - 1; m >= 0; --m) {
      const C<T> cm = {mu[m] * T(kInvFact.v[m]), T(0)};
      fs = cfma(fs, C<T>{tr, ti}, cm);      // sum (tau)^m mu_m / m!
      gs = cfma(gs, C<T>{-tr, -ti}, cm);    // sum (-tau)^m mu_m / m!
    }
    // exp(-tau h) for h = hf, hg: |tau| h <= r, so the series to degree KK >= K
    // is exact to the unit roundoff (the table holds degrees up to kTaylorMax;
    // beyond, the library functions); the tile's factor A = exp(-tau (hf + hg)).
    C<T> ef = {T(0), T(0)}, eg = {T(0), T(0)};
    if constexpr (KK <= kTaylorMax) {
#pragma unroll
      for (int m = KK; m >= 0; --m) {
        const T c_re = T(md.coef_re[k][m]), c_im = T(md.coef_im[k][m]);
        ef.re = fma(ef.re, g.hf, c_re);
        ef.im = fma(ef.im, g.hf, c_im);
        eg.re = fma(eg.re, g.hg, c_re);
        eg.im = fma(eg.im, g.hg, c_im);
      }
    } else {
      ef = exp_neg_general<T>(tr, ti, g.hf);
      eg = exp_neg_general<T>(tr, ti, g.hg);
    }
    const C<T> a = cmul(ef, eg);
    const C<T> f = cmul(ef, fs);
    const C<T> gg = cmul(eg, gs);
    T* o = out + k * kAggStride;
    o[0] = a.re; o[1] = a.im;
    o[2] = f.re; o[3] = f.im;
    o[4] = gg.re; o[5] = gg.im;
    o[6] = ef.re; o[7] = ef.im;
    o[8] = eg.re; o[9] = eg.im;
  }
}

// Strengths: read from bs, or (src set) gathered from src by merged id and
// stored to b_store.
template <class T, int NM>
__global__ __launch_bounds__(256) void k_wreduce(const void* keys0, const void* keys1,
                                                 const PassInfo* __restrict__ pass,
                                                 const T* __restrict__ bs,
                                                 const T* __restrict__ src, uint32_t n_src,
                                                 const uint32_t* __restrict__ ids,
                                                 T* __restrict__ b_store, int64_t P,
                                                 int64_t tiles, int vec, Modes md,
                                                 T* __restrict__ agg,
                                                 int32_t* __restrict__ tile_k) {
  const KeyView<T> keys = key_view<T>(keys0, keys1, pass);
  const int lane = threadIdx.x % kWave;
  const int64_t tile = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  if (tile >= tiles) return;
  const int64_t t0 = tile * kWTile;
  T zc[kScanChunk], bc[kScanChunk], dz[kScanChunk], sc[kScanChunk];
  if (src)
    load_gather(keys.z, ids, src, n_src, b_store, t0 + lane * kScanChunk, P, vec != 0, zc, bc);
  else
    load_chunk(keys.z, bs, t0 + lane * kScanChunk, P, vec != 0, zc, bc);
  const TileGeo<T> g = tile_geometry(keys.z, t0, P, lane, zc, dz, sc);
  const int K = moment_count(T(md.tau_abs_max) * (g.hf > g.hg ? g.hf : g.hg));
  if (lane == 0) tile_k[tile] = K;
  T* out = agg + (size_t)tile * NM * kAggStride;
  if (K >= 0) {
    switch (k_class(K)) {
      case 0: reduce_moments<T, NM, kKSteps[0]>(md, bc, sc, g, lane, out); break;
      case 1: reduce_moments<T, NM, kKSteps[1]>(md, bc, sc, g, lane, out); break;
      case 2: reduce_moments<T, NM, kKSteps[2]>(md, bc, sc, g, lane, out); break;
      case 3: reduce_moments<T, NM, kKSteps[3]>(md, bc, sc, g, lane, out); break;
      case 4: reduce_moments<T, NM, kKSteps[4]>(md, bc, sc, g, lane, out); break;
      case 5: reduce_moments<T, NM, kKSteps[5]>(md, bc, sc, g, lane, out); break;
      default: reduce_moments<T, NM, kKSteps[6]>(md, bc, sc, g, lane, out); break;
    }
    return;
  }
  // Wide tile: each lane folds its chunk's recurrences, then the lanes' maps
  // are composed in order.
#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    C<T> ex[kScanChunk];
    mode_exps(md, k, dz, g.dzmax, ex);
    Seg<T> s;
    s.a = ex[0];
    s.f = {bc[0], T(0)};
#pragma unroll
    for (int j = 1; j < kScanChunk; ++j) {
      s.a = cmul(s.a, ex[j]);
      s.f = cfma(ex[j], s.f, C<T>{bc[j], T(0)});
    }
    s.g = {T(0), T(0)};
#pragma unroll
    for (int j = kScanChunk - 1; j >= 0; --j) s.g = cmul(ex[j], cadd(s.g, C<T>{bc[j], T(0)}));
    Seg<T> pf, sb;
    wave_scans(s, lane, pf, sb);
    T* o = out + k * kAggStride;
    if (lane == kWave - 1) {
      o[0] = pf.a.re; o[1] = pf.a.im;
      o[2] = pf.f.re; o[3] = pf.f.im;
    }
    if (lane == 0) {
      o[4] = sb.g.re; o[5] = sb.g.im;
    }
  }
}

// Scatter of one chunk's results: point j feeds output id_j - t_lo when that
// is below t_n (the unsigned compare keeps every write in bounds).
template <class T>
__device__ __forceinline__ void scatter_chunk(const ScanOut<T>& out, const uint32_t* ids,
                                              const T* acc) {
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    const uint32_t o = ids[j] - out.t_lo;
    if (o < out.t_n) out.val[o] = acc[j];
  }
}

// Both sweeps of a chunk for one mode from the values entering it: h+ at the
// point before the chunk (h) and h- at its last point (g); Re(omega (h+ + h-))
// is added to acc.
template <class T>
__device__ __forceinline__ void sweeps(const C<T>* ex, const T* bc, C<T> h, C<T> g, T om_re,
                                       T om_im, T* acc) {
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    h = cfma(ex[j], h, C<T>{bc[j], T(0)});
    acc[j] = fma(om_re, h.re, fma(-om_im, h.im, acc[j]));
  }
#pragma unroll
  for (int j = kScanChunk - 1; j >= 0; --j) {
    acc[j] = fma(om_re, g.re, fma(-om_im, g.im, acc[j]));
    g = cmul(ex[j], cadd(g, C<T>{bc[j], T(0)}));
  }
}

// ---------------------------------------------------------------------------
// k_wfinal_fast: tiles with at most kFastMoments moments.  The value entering
// each lane's chunk comes from the moments of the tile's other chunks about
// the tile centre c:
//   h+ before the chunk  = E_f (CF eG + sum_m tau^m P_m / m!),    E_f = exp(-tau (z_s - c)),
//   h- at its last point = E_b (CB eF + sum_m (-tau)^m S_m / m!), E_b = exp(-tau (c - z_e)),
// with P_m / S_m the moments of the tile's points before / after the chunk
// (exclusive prefix and suffix over the lanes), CF, CB the tile carries and
// eF = exp(-tau hf), eG = exp(-tau hg) from k_wreduce.
// ---------------------------------------------------------------------------
template <class T, int NM, int KK>
__device__ __forceinline__ void final_fast_body(const Modes& md, const T* dz, const T* bc,
                                                const T* sc, const TileGeo<T>& g, int lane,
                                                const T* __restrict__ ag,
                                                const T* __restrict__ cr, T* acc) {
  // Prefix (before the chunk) and suffix (after it) moments, divided by m!.
  T pre[KK + 1], suf[KK + 1];
  {
    T pw[kScanChunk];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) pw[j] = bc[j];
#pragma unroll
    for (int m = 0; m <= KK; ++m) {
      T nu = T(0);
#pragma unroll
      for (int j = 0; j < kScanChunk; ++j) {
        nu += pw[j];
        pw[j] *= sc[j];
      }
      const T inc = wave_inclusive_sum(nu);
      const T tot = lane_value(inc, kWave - 1);
      const T f = T(kInvFact.v[m]);
      pre[m] = (inc - nu) * f;   // the lanes before this one
      suf[m] = (tot - inc) * f;  // the lanes after it
    }
  }
  const T xf = g.zs - g.c;
  const T xb = g.c - g.ze;
#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
    C<T> ef = {T(0), T(0)}, eb = {T(0), T(0)};
    C<T> fs = {pre[KK], T(0)}, gs = {suf[KK], T(0)};
#pragma unroll
    for (int m = KK; m >= 0; --m) {
      const T c_re = T(md.coef_re[k][m]), c_im = T(md.coef_im[k][m]);
      ef.re = fma(ef.re, xf, c_re);
      ef.im = fma(ef.im, xf, c_im);
      eb.re = fma(eb.re, xb, c_re);
      eb.im = fma(eb.im, xb, c_im);
      if (m < KK) {
        fs = cfma(fs, C<T>{tr, ti}, C<T>{pre[m], T(0)});
        gs = cfma(gs, C<T>{-tr, -ti}, C<T>{suf[m], T(0)});
      }
    }
    const T* a = ag + k * kAggStride;
    const T* c = cr + k * 4;
    const C<T> tf = cfma(C<T>{c[0], c[1]}, C<T>{a[8], a[9]}, fs);   // CF eG + fs
    const C<T> tb = cfma(C<T>{c[2], c[3]}, C<T>{a[6], a[7]}, gs);   // CB eF + gs
    C<T> ex[kScanChunk];
    mode_exps(md, k, dz, g.dzmax, ex);
    sweeps(ex, bc, cmul(ef, tf), cmul(eb, tb), T(md.om_re[k]), T(md.om_im[k]), acc);
  }
}

// Tiles of the rare classes (more moments, or wide) are looked for by waves
// that each test kRareSpan tiles spread over the whole sequence (tile
// w + j * waves for lane j): when there are none, the kernel costs one load
// per wave instead of one wave per tile, and where there are many (clustered
// data) they are shared evenly between the waves.
constexpr int kRareSpan = 4;

__host__ __device__ __forceinline__ int64_t rare_waves(int64_t tiles) {
  return (tiles + kRareSpan - 1) / kRareSpan;
}

// Calls body(tile, K) for every tile whose count K satisfies is_mine(K).
template <class Pred, class Body>
__device__ __forceinline__ void for_rare_tiles(const int32_t* __restrict__ tile_k, int64_t tiles,
                                               Pred is_mine, Body body) {
  const int lane = threadIdx.x % kWave;
  const int64_t nw = rare_waves(tiles);
  const int64_t w = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
  if (w >= nw) return;
  const int64_t t = w + (int64_t)lane * nw;
  const bool in = lane < kRareSpan && t < tiles;
  const int Kl = in ? tile_k[t] : 0;
  uint64_t todo = __ballot(in && is_mine(Kl));
#pragma unroll 1
  while (todo) {
    const int j = __builtin_ctzll(todo);
    todo &= todo - 1;
    // Tile and count as lane values (a shuffle): taken as wave-uniform, they
    // led the compiler to a schedule with ~90 more registers per lane.
    const int jv = __shfl(j, lane);
    body(w + (int64_t)jv * nw, __shfl(Kl, jv));
  }
}

// One tile of k_wfinal_fast.
template <class T, int NM, int KMAX>
__device__ __forceinline__ void wfinal_fast_tile(const KeyView<T>& keys,
                                                 const T* __restrict__ bs,
                                                 const uint32_t* __restrict__ ids, int64_t P,
                                                 int vec, const Modes& md,
                                                 const T* __restrict__ agg,
                                                 const T* __restrict__ carry, ScanOut<T> out,
                                                 int64_t tile, int K) {
  const int lane = threadIdx.x % kWave;
  const int64_t t0 = tile * kWTile;
  const int64_t base = t0 + lane * kScanChunk;
  T zc[kScanChunk], bc[kScanChunk], dz[kScanChunk], sc[kScanChunk], acc[kScanChunk];
  load_chunk(keys.z, bs, base, P, vec != 0, zc, bc);
  const TileGeo<T> g = tile_geometry(keys.z, t0, P, lane, zc, dz, sc);
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) acc[j] = T(0);
  const T* ag = agg + (size_t)tile * NM * kAggStride;
  const T* cr = carry + (size_t)tile * NM * 4;
  if constexpr (KMAX == kKSteps[2]) {
    switch (k_class(K)) {
      case 0: final_fast_body<T, NM, kKSteps[0]>(md, dz, bc, sc, g, lane, ag, cr, acc); break;
      case 1: final_fast_body<T, NM, kKSteps[1]>(md, dz, bc, sc, g, lane, ag, cr, acc); break;
      default: final_fast_body<T, NM, kKSteps[2]>(md, dz, bc, sc, g, lane, ag, cr, acc); break;
    }
  } else {
    if (k_class(K) == 3)
      final_fast_body<T, NM, kKSteps[3]>(md, dz, bc, sc, g, lane, ag, cr, acc);
    else
      final_fast_body<T, NM, kKSteps[4]>(md, dz, bc, sc, g, lane, ag, cr, acc);
  }
  uint32_t ic[kScanChunk];   // loaded last: not live during the sweeps
  load_ids(ids, base, P, vec != 0, ic);
  scatter_chunk(out, ic, acc);
}

// Two instantiations: moment counts up to kKSteps[2] (the usual case: one
// wave per tile) and the larger ones up to kFastMoments (rare: see
// for_rare_tiles), so that the common kernel keeps fewer registers (its
// moment arrays are shorter) and runs more waves per SIMD.
template <class T, int NM, int KMAX>
__global__ __launch_bounds__(256) void k_wfinal_fast(const void* keys0, const void* keys1,
                                                     const PassInfo* __restrict__ pass,
                                                     const T* __restrict__ bs,
                                                     const uint32_t* __restrict__ ids, int64_t P,
                                                     int64_t tiles, int vec, Modes md,
                                                     const T* __restrict__ agg,
                                                     const T* __restrict__ carry,
                                                     const int32_t* __restrict__ tile_k,
                                                     ScanOut<T> out) {
  const KeyView<T> keys = key_view<T>(keys0, keys1, pass);
  if constexpr (KMAX == kKSteps[2]) {
    const int64_t tile = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (tile >= tiles) return;
    const int K = tile_k[tile];
    if (K < 0 || K > KMAX) return;   // another kernel's tile
    wfinal_fast_tile<T, NM, KMAX>(keys, bs, ids, P, vec, md, agg, carry, out, tile, K);
  } else {
    for_rare_tiles(tile_k, tiles, [](int K) { return K > kKSteps[2] && K <= KMAX; },
                   [&](int64_t tile, int K) {
                     wfinal_fast_tile<T, NM, KMAX>(keys, bs, ids, P, vec, md, agg, carry, out,
                                                   tile, K);
                   });
  }
}

// ---------------------------------------------------------------------------
// k_wfinal: the other tiles.  Per mode: the lanes' chunk maps, their inclusive
// prefix (forward) and suffix (backward) over the wave, the tile carries, the
// sweeps.
// ---------------------------------------------------------------------------

// One tile of k_wfinal.
template <class T, int NM>
__device__ __forceinline__ void wfinal_tile(const KeyView<T>& keys, const T* __restrict__ bs,
                                            const uint32_t* __restrict__ ids, int64_t P, int vec,
                                            const Modes& md, const T* __restrict__ carry,
                                            ScanOut<T> out, int64_t tile) {
  const int lane = threadIdx.x % kWave;
  const int64_t t0 = tile * kWTile;
  const int64_t base = t0 + lane * kScanChunk;
  T zc[kScanChunk], bc[kScanChunk], dz[kScanChunk], sc[kScanChunk], acc[kScanChunk];
  uint32_t ic[kScanChunk];
  load_chunk(keys.z, bs, base, P, vec != 0, zc, bc);
  load_ids(ids, base, P, vec != 0, ic);
  const TileGeo<T> g = tile_geometry(keys.z, t0, P, lane, zc, dz, sc);
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) acc[j] = T(0);
#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    C<T> ex[kScanChunk];
    mode_exps(md, k, dz, g.dzmax, ex);
    Seg<T> s;
    s.a = ex[0];
    s.f = {bc[0], T(0)};
#pragma unroll
    for (int j = 1; j < kScanChunk; ++j) {
      s.a = cmul(s.a, ex[j]);
      s.f = cfma(ex[j], s.f, C<T>{bc[j], T(0)});
    }
    s.g = {T(0), T(0)};
#pragma unroll
    for (int j = kScanChunk - 1; j >= 0; --j) s.g = cmul(ex[j], cadd(s.g, C<T>{bc[j], T(0)}));
    Seg<T> pf, sb;
    wave_scans(s, lane, pf, sb);
    const T* cr = carry + ((size_t)tile * NM + k) * 4;
    C<T> cf = {cr[0], cr[1]};
    C<T> cb = {cr[2], cr[3]};
    // exclusive lane prefix / suffix
    Seg<T> xl, xr;
    xl.a.re = shfl_up(pf.a.re, 1); xl.a.im = shfl_up(pf.a.im, 1);
    xl.f.re = shfl_up(pf.f.re, 1); xl.f.im = shfl_up(pf.f.im, 1);
    xr.a.re = shfl_down(sb.a.re, 1); xr.a.im = shfl_down(sb.a.im, 1);
    xr.g.re = shfl_down(sb.g.re, 1); xr.g.im = shfl_down(sb.g.im, 1);
    if (lane > 0) cf = cfma(xl.a, cf, xl.f);
    if (lane < kWave - 1) cb = cfma(xr.a, cb, xr.g);
    sweeps(ex, bc, cf, cb, T(md.om_re[k]), T(md.om_im[k]), acc);
  }
  scatter_chunk(out, ic, acc);
}

template <class T, int NM>
__global__ __launch_bounds__(256) void k_wfinal(const void* keys0, const void* keys1,
                                                const PassInfo* __restrict__ pass,
                                                const T* __restrict__ bs,
                                                const uint32_t* __restrict__ ids, int64_t P,
                                                int64_t tiles, int vec, Modes md,
                                                const T* __restrict__ carry,
                                                const int32_t* __restrict__ tile_k,
                                                ScanOut<T> out) {
  const KeyView<T> keys = key_view<T>(keys0, keys1, pass);
  // the tiles that k_wfinal_fast does not take
  for_rare_tiles(tile_k, tiles, [](int K) { return K < 0 || K > kFastMoments; },
                 [&](int64_t tile, int) { wfinal_tile<T, NM>(keys, bs, ids, P, vec, md, carry, out,
                                                            tile); });
}

template <class T>
__global__ void k_fill_zero(T* __restrict__ u, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) u[i] = T(0);
}

template <class T>
hipError_t carry_tiles(const Workspace& w, int64_t tiles, int nq, hipStream_t s) {
  return launch_carries<T>(AggMaps<T>{(const T*)w.agg, nq}, tiles, nq, (T*)w.chunk_agg,
                           (T*)w.chunk_carry, (T*)w.carry, s);
}

// 16-byte loads of a lane's chunk need 16-byte aligned arrays.
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <class T, int NM>
hipError_t scan_nm(const Workspace& w, const Modes& md, int64_t P, const T* b_in, const T* src,
                   uint32_t n_src, const ScanOut<T>& out, hipStream_t s, Timeline* tl) {
  const int64_t tiles = (P + kWTile - 1) / kWTile;
  const dim3 grid((unsigned)((tiles + 3) / 4));
  // With src the reduce stores the gathered strengths to w.b for the later kernels.
  const T* b = src ? (const T*)w.b : b_in;
  const int vec = aligned16(w.keys[0]) && aligned16(w.keys[1]) && aligned16(b) &&
                  aligned16(w.ids);
  hipLaunchKernelGGL((k_wreduce<T, NM>), grid, dim3(256), 0, s, w.keys[0], w.keys[1], w.pass,
                     src ? nullptr : b, src, n_src, (const uint32_t*)w.ids, (T*)w.b, P, tiles, vec,
                     md, (T*)w.agg, w.tile_k);
  tl->mark(s);
  (void)carry_tiles<T>(w, tiles, NM, s);
  tl->mark(s);
  hipLaunchKernelGGL((k_wfinal_fast<T, NM, kKSteps[2]>), grid, dim3(256), 0, s, w.keys[0],
                     w.keys[1], w.pass, b, w.ids, P, tiles, vec, md, (const T*)w.agg,
                     (const T*)w.carry, w.tile_k, out);
  // The rare classes: one wave per kRareSpan tiles.
  const dim3 rare_grid((unsigned)((rare_waves(tiles) + 3) / 4));
  hipLaunchKernelGGL((k_wfinal_fast<T, NM, kFastMoments>), rare_grid, dim3(256), 0, s, w.keys[0],
                     w.keys[1], w.pass, b, w.ids, P, tiles, vec, md, (const T*)w.agg,
                     (const T*)w.carry, w.tile_k, out);
  hipLaunchKernelGGL((k_wfinal<T, NM>), rare_grid, dim3(256), 0, s, w.keys[0], w.keys[1], w.pass,
                     b, w.ids, P, tiles, vec, md, (const T*)w.carry, w.tile_k, out);
  tl->mark(s);
  return hipGetLastError();
}

template <class T>
__global__ __launch_bounds__(256) void k_gather(const uint32_t* __restrict__ ids, int64_t P,
                                                uint32_t lo, uint32_t n, const T* __restrict__ wts,
                                                T* __restrict__ b) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; p < P; p += stride) {
    const uint32_t o = ids[p] - lo;
    b[p] = o < n ? wts[o] : T(0);
  }
}

}  // namespace

template <class T>
hipError_t scan_points(const Workspace& w, const Modes& md, int64_t P, const T* b, const T* src,
                       uint32_t n_src, const ScanOut<T>& out, hipStream_t s, Timeline* tl) {
  if (!out.val || out.der) return hipErrorInvalidValue;   // the adjoint has its own kernels
  switch (md.n) {
    case 1: return scan_nm<T, 1>(w, md, P, b, src, n_src, out, s, tl);
    case 2: return scan_nm<T, 2>(w, md, P, b, src, n_src, out, s, tl);
    case 3: return scan_nm<T, 3>(w, md, P, b, src, n_src, out, s, tl);
    case 4: return scan_nm<T, 4>(w, md, P, b, src, n_src, out, s, tl);
    case 5: return scan_nm<T, 5>(w, md, P, b, src, n_src, out, s, tl);
    case 6: return scan_nm<T, 6>(w, md, P, b, src, n_src, out, s, tl);
    case 7: return scan_nm<T, 7>(w, md, P, b, src, n_src, out, s, tl);
    default: return hipErrorInvalidValue;
  }
}

template <class T>
hipError_t gather_strengths(const Workspace& w, int64_t P, uint32_t lo, uint32_t n, const T* wts,
                            T* b, hipStream_t s) {
  int64_t blocks = (P + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_gather<T>, dim3((unsigned)blocks), dim3(256), 0, s, w.ids, P, lo, n, wts, b);
  return hipGetLastError();
}

template <class T>
hipError_t fill_zero(T* u, int64_t n, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_zero<T>, dim3((unsigned)blocks), dim3(256), 0, s, u, n);
  return hipGetLastError();
}

template hipError_t scan_points<double>(const Workspace&, const Modes&, int64_t, const double*,
                                        const double*, uint32_t, const ScanOut<double>&,
                                        hipStream_t, Timeline*);
template hipError_t scan_points<float>(const Workspace&, const Modes&, int64_t, const float*,
                                       const float*, uint32_t, const ScanOut<float>&, hipStream_t,
                                       Timeline*);
template hipError_t gather_strengths<double>(const Workspace&, int64_t, uint32_t, uint32_t,
                                             const double*, double*, hipStream_t);
template hipError_t gather_strengths<float>(const Workspace&, int64_t, uint32_t, uint32_t,
                                            const float*, float*, hipStream_t);
template hipError_t fill_zero<double>(double*, int64_t, hipStream_t);
template hipError_t fill_zero<float>(float*, int64_t, hipStream_t);

}  // namespace fgt
