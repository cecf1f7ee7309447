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
// The same sweeps give the x-derivative of the transform: h+ holds the sources
// to the left (sign +1), h- those to the right (sign -1), so
//     u'_p = sum_k Re(-tau_k omega_k (h+_p - h-_p)).
// The gradients of L = sum_i g_i u_i are such scans with the roles of sources
// and targets kept (dL/dx) or swapped (dL/dalpha, dL/dy: strengths g at the
// targets, outputs at the sources).
//
// A segment [s, e) of the sequence acts on the two recurrences as
//     h+_{e-1} = A h+_{s-1} + F,          h-_{s-1} = A h-_{e-1} + G,
//     A = prod_{p in seg} e_p = exp(-tau (z_{e-1} - z_{s-1})),
//     F = sum_{q in seg} b_q exp(-tau (z_{e-1} - z_q)),   G = sum_{q in seg} b_q exp(-tau (z_q - z_{s-1})),
// and segments compose associatively:  (A1,F1,G1).(A2,F2,G2) = (A1 A2, A2 F1 + F2, G1 + A1 G2).
//
// Three kernels, reduce-then-scan over tiles of kScanTile points:
//   k_reduce   one wave per tile: the tile's (A, F, G) for every mode.  When the
//              tile is short on the decay scale (|tau| times its half-width small)
//              the sums come from mode-independent power moments of the strengths
//              about the tile centre c:  sum_q b_q exp(+-tau (z_q - c)) =
//              sum_m (+-tau)^m mu_m / m!,  mu_m = sum_q b_q (z_q - c)^m;
//              otherwise from the recurrences themselves.
//   k_carry_* per mode: exclusive prefix of F and suffix of G over tiles.
//   k_final    per tile: chunk -> wave -> tile scans of both recurrences with
//              the carries, sweeps, mode reduction, scatter to the outputs.
#include "fgt_device.h"

namespace fgt {
namespace {

// ---------------------------------------------------------------------------
// k_reduce: (A, F, G) of every tile and mode.  One wave per tile.
// ---------------------------------------------------------------------------
template <class T, int NM>
__global__ __launch_bounds__(kWave) void k_reduce(const void* keys0, const void* keys1,
                                                  const PassInfo* __restrict__ pass,
                                                  const T* __restrict__ bs, int64_t P, Modes md,
                                                  T* __restrict__ agg,
                                                  int32_t* __restrict__ tile_k) {
  const KeyView<T> keys = key_view<T>(keys0, keys1, pass);
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t t0 = tile * kScanTile;
  const int n = (int)((P - t0) < kScanTile ? (P - t0) : kScanTile);
  const T zfirst = keys(t0);
  const T zprev = t0 > 0 ? keys(t0 - 1) : zfirst;
  const T zlast = keys(t0 + n - 1);
  // Centre c and the exact distances to the tile's outer reference points.
  const T c = zprev + (zlast - zprev) * T(0.5);
  const T hf = zlast - c;
  const T hg = c - zprev;
  const T span = zlast - zprev;
  const T r = T(md.tau_abs_max) * (hf > hg ? hf : hg);

  // Number of moments: the series tail r^{K+1}/(K+1)! e^r must be below the unit roundoff.
  int K = 0;
  {
    const T er = exp_t(r);
    T t = r;
    while (t * er > T(Prec<T>::kUnit) && K < kMomentMax) {
      ++K;
      t *= r / T(K + 1);
    }
    if (t * er > T(Prec<T>::kUnit)) K = -1;   // too wide: use the recurrences
  }
  if (lane == 0) tile_k[tile] = K;

  if (K >= 0) {
    T mu[kMomentMax + 1];
#pragma unroll
    for (int m = 0; m <= kMomentMax; ++m) mu[m] = T(0);
    // The lane's points in order, kGrp at a time with all their loads issued
    // before any is used.  The loads are nontemporal: the final kernel reads
    // these arrays again, but they are far larger than the caches.
    constexpr int kGrp = 8;
#pragma unroll 1
    for (int g0 = 0; g0 < kScanTile / kWave; g0 += kGrp) {
      T zg[kGrp], bg[kGrp];
#pragma unroll
      for (int i = 0; i < kGrp; ++i) {
        const int e = lane + (g0 + i) * kWave;
        const bool in = e < n;
        zg[i] = in ? __builtin_nontemporal_load(&keys.z[t0 + e]) : c;
        bg[i] = in ? __builtin_nontemporal_load(&bs[t0 + e]) : T(0);
      }
#pragma unroll
      for (int i = 0; i < kGrp; ++i) {
        const T s = zg[i] - c;
        T pw = bg[i];
        mu[0] += pw;
#pragma unroll
        for (int m = 1; m <= kMomentMax; ++m) {
          if (m <= K) {
            pw *= s;
            mu[m] += pw;
          }
        }
      }
    }
    // Butterfly sums: every lane ends with the same, order-fixed totals (the
    // moments' shuffles interleaved).
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
#pragma unroll
      for (int m = 0; m <= kMomentMax; ++m)
        if (m <= K) mu[m] += shfl_xor(mu[m], o);
    }
    if (lane < NM) {
      const int k = lane;
      const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
      T top = T(0);
#pragma unroll
      for (int m = 0; m <= kMomentMax; ++m)
        if (m == K) top = mu[m];
      C<T> fs = {top * T(kInvFact.v[K]), T(0)};
      C<T> gs = fs;
#pragma unroll
      for (int m = kMomentMax - 1; m >= 0; --m) {
        if (m < K) {
          const C<T> cm = {mu[m] * T(kInvFact.v[m]), T(0)};
          fs = cfma(fs, C<T>{tr, ti}, cm);      // sum (tau)^m mu_m / m!
          gs = cfma(gs, C<T>{-tr, -ti}, cm);    // sum (-tau)^m mu_m / m!
        }
      }
      const C<T> ef = exp_neg_general<T>(tr, ti, hf);
      const C<T> eg = exp_neg_general<T>(tr, ti, hg);
      const C<T> a = exp_neg_general<T>(tr, ti, span);
      const C<T> f = cmul(ef, fs);
      const C<T> g = cmul(eg, gs);
      T* o = agg + ((size_t)tile * NM + k) * kAggStride;
      o[0] = a.re; o[1] = a.im;
      o[2] = f.re; o[3] = f.im;
      o[4] = g.re; o[5] = g.im;
      o[6] = ef.re; o[7] = ef.im;
      o[8] = eg.re; o[9] = eg.im;
    }
    return;
  }

  // Wide tile: fold the recurrences over kPer consecutive points per lane,
  // then compose the lanes' maps in order.
  constexpr int kPer = kScanTile / kWave;
  const int e0 = lane * kPer;
  const int cnt = n - e0 < 0 ? 0 : (n - e0 < kPer ? n - e0 : kPer);
#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
    Seg<T> s = seg_identity<T>();
    // forward map (A, F)
    T zl = e0 == 0 ? zprev : (cnt > 0 ? keys(t0 + e0 - 1) : zlast);
    for (int j = 0; j < cnt; ++j) {
      const T zj = keys(t0 + e0 + j);
      const C<T> ex = exp_neg_general<T>(tr, ti, zj - zl);
      s.a = cmul(s.a, ex);
      s.f = cfma(ex, s.f, C<T>{bs[t0 + e0 + j], T(0)});
      zl = zj;
    }
    // backward map G, last point first
    C<T> g = {T(0), T(0)};
    for (int j = cnt - 1; j >= 0; --j) {
      const T zj = keys(t0 + e0 + j);
      const T zb = (e0 + j == 0) ? zprev : keys(t0 + e0 + j - 1);
      const C<T> ex = exp_neg_general<T>(tr, ti, zj - zb);
      g = cmul(ex, cadd(g, C<T>{bs[t0 + e0 + j], T(0)}));
    }
    s.g = g;
    Seg<T> pf = s, sb = s;
    for (int o = 1; o < kWave; o <<= 1) {
      Seg<T> l, rr;
      l.a.re = shfl_up(pf.a.re, o); l.a.im = shfl_up(pf.a.im, o);
      l.f.re = shfl_up(pf.f.re, o); l.f.im = shfl_up(pf.f.im, o);
      if (lane >= o) {
        pf.f = cfma(pf.a, l.f, pf.f);
        pf.a = cmul(l.a, pf.a);
      }
      rr.a.re = shfl_down(sb.a.re, o); rr.a.im = shfl_down(sb.a.im, o);
      rr.g.re = shfl_down(sb.g.re, o); rr.g.im = shfl_down(sb.g.im, o);
      if (lane + o < kWave) {
        sb.g = cfma(sb.a, rr.g, sb.g);
        sb.a = cmul(sb.a, rr.a);
      }
    }
    T* o = agg + ((size_t)tile * NM + k) * kAggStride;
    if (lane == kWave - 1) {
      o[0] = pf.a.re; o[1] = pf.a.im;
      o[2] = pf.f.re; o[3] = pf.f.im;
    }
    if (lane == 0) {
      o[4] = sb.g.re; o[5] = sb.g.im;
    }
  }
}

// ---------------------------------------------------------------------------
// k_final: both sweeps with the carries, mode reduction, scatter.
// ---------------------------------------------------------------------------
template <class T>
struct Staged {
  T z[kScanTile + kScanTile / kScanChunk];
  T b[kScanTile + kScanTile / kScanChunk];
  uint32_t id[kScanTile + kScanTile / kScanChunk];
};

// Scatter of one chunk's results (see ScanOut).
template <class T, int OUT>
__device__ __forceinline__ void scatter_chunk(const ScanOut<T>& out, const uint32_t* ids,
                                              const T* acc, const T* dacc) {
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    const uint32_t o = ids[j] - out.t_lo;
    if (o < out.t_n) {
      if (OUT & kOutVal) out.val[o] = acc[j];
      if (OUT & kOutDer) out.der[o] = out.scale ? dacc[j] * out.scale[o] : dacc[j];
    }
  }
}

__device__ __forceinline__ int lds_pos(int e) { return e + e / kScanChunk; }

template <class T, int NM, int OUT>
__global__ __launch_bounds__(kScanThreads) void k_final(const void* keys0, const void* keys1,
                                                        const PassInfo* __restrict__ pass,
                                                        const T* __restrict__ bs,
                                                        const uint32_t* __restrict__ ids,
                                                        int64_t P, Modes md,
                                                        const T* __restrict__ carry,
                                                        const int32_t* __restrict__ tile_k,
                                                        ScanOut<T> out) {
  {
    const int K = tile_k[blockIdx.x];
    if (K >= 0 && K <= kFastMoments) return;   // handled by k_final_fast
  }
  const KeyView<T> keys = key_view<T>(keys0, keys1, pass);
  __shared__ Staged<T> st;
  __shared__ Seg<T> wtot[NM][kScanWaves][2];   // per wave: [0] forward total, [1] backward total
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int64_t tile = blockIdx.x;
  const int64_t t0 = tile * kScanTile;

  {
    // All of this thread's loads are issued before any is used; they are the
    // last reads of the sorted points in this call, so they are nontemporal.
    constexpr int R = kScanTile / kScanThreads;
    T zr[R], br[R];
    uint32_t sr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t p = t0 + tid + r * kScanThreads;
      const bool in = p < P;
      zr[r] = in ? __builtin_nontemporal_load(&keys.z[p]) : T(0);
      br[r] = in ? __builtin_nontemporal_load(&bs[p]) : T(0);
      sr[r] = in ? __builtin_nontemporal_load(&ids[p]) : kNoSlot;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = lds_pos(tid + r * kScanThreads);
      st.z[q] = zr[r];
      st.b[q] = br[r];
      st.id[q] = sr[r];
    }
  }
  T zprev = T(0);
  if (tid == 0) zprev = t0 > 0 ? keys(t0 - 1) : T(0);
  __syncthreads();

  // This thread's chunk: gaps dz_j = z_j - z_{j-1} and strengths b_j.
  const int e0 = tid * kScanChunk;
  T dz[kScanChunk], bb[kScanChunk];
  T dzmax = T(0);
  {
    const int64_t valid = P - t0;
    T zl;
    if (tid == 0)
      zl = t0 > 0 ? zprev : st.z[lds_pos(0)];
    else
      zl = st.z[lds_pos(e0 - 1)];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      const int e = e0 + j;
      const T zj = st.z[lds_pos(e)];
      dz[j] = (e < valid) ? zj - zl : T(0);
      bb[j] = st.b[lds_pos(e)];
      zl = (e < valid) ? zj : zl;
      dzmax = dz[j] > dzmax ? dz[j] : dzmax;
    }
  }
  // Largest gap in the wave: sets the Taylor degree of the mode exponentials.
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const T other = shfl_xor(dzmax, o);
    dzmax = other > dzmax ? other : dzmax;
  }

  T acc[kScanChunk], dacc[kScanChunk];
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    acc[j] = T(0);
    dacc[j] = T(0);
  }

#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
    const T om_re = T(md.om_re[k]), om_im = T(md.om_im[k]);
    const T dm_re = T(md.dom_re[k]), dm_im = T(md.dom_im[k]);
    // Degree D: smallest with (|tau| dzmax)^{D+1}/(D+1)! below the unit roundoff.
    const double rr = md.tau_abs[k] * (double)dzmax;
    int D = kTaylorMax;
#pragma unroll
    for (int d = kTaylorMax; d >= 1; --d)
      if (rr <= md.taylor_thr[d]) D = d;
    const T dz_lim = T(md.dz_lim[k]);

    // e_j = sum_{m<=D} (-tau)^m dz_j^m / m!  (Horner in the real variable dz)
    C<T> ex[kScanChunk];
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
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j)
      if (dz[j] > dz_lim) ex[j] = exp_neg_general<T>(tr, ti, dz[j]);

    // Chunk map.
    Seg<T> s;
    s.a = ex[0];
    s.f = {bb[0], T(0)};
#pragma unroll
    for (int j = 1; j < kScanChunk; ++j) {
      s.a = cmul(s.a, ex[j]);
      s.f = cfma(ex[j], s.f, C<T>{bb[j], T(0)});
    }
    s.g = {T(0), T(0)};
#pragma unroll
    for (int j = kScanChunk - 1; j >= 0; --j) s.g = cmul(ex[j], cadd(s.g, C<T>{bb[j], T(0)}));

    // Inclusive forward scan over lanes (prefix) and backward scan (suffix).
    Seg<T> pf = s, sb = s;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      Seg<T> l;
      l.a.re = shfl_up(pf.a.re, o); l.a.im = shfl_up(pf.a.im, o);
      l.f.re = shfl_up(pf.f.re, o); l.f.im = shfl_up(pf.f.im, o);
      if (lane >= o) {
        pf.f = cfma(pf.a, l.f, pf.f);
        pf.a = cmul(l.a, pf.a);
      }
      Seg<T> r;
      r.a.re = shfl_down(sb.a.re, o); r.a.im = shfl_down(sb.a.im, o);
      r.g.re = shfl_down(sb.g.re, o); r.g.im = shfl_down(sb.g.im, o);
      if (lane + o < kWave) {
        sb.g = cfma(sb.a, r.g, sb.g);
        sb.a = cmul(sb.a, r.a);
      }
    }
    if (lane == kWave - 1) wtot[k][wave][0] = pf;
    if (lane == 0) wtot[k][wave][1] = sb;
    __syncthreads();

    const T* cr = carry + ((size_t)tile * NM + k) * 4;
    C<T> cf = {cr[0], cr[1]};
    C<T> cb = {cr[2], cr[3]};
    for (int w = 0; w < wave; ++w) cf = cfma(wtot[k][w][0].a, cf, wtot[k][w][0].f);
    for (int w = kScanWaves - 1; w > wave; --w) cb = cfma(wtot[k][w][1].a, cb, wtot[k][w][1].g);
    // exclusive lane prefix / suffix
    Seg<T> xl, xr;
    xl.a.re = shfl_up(pf.a.re, 1); xl.a.im = shfl_up(pf.a.im, 1);
    xl.f.re = shfl_up(pf.f.re, 1); xl.f.im = shfl_up(pf.f.im, 1);
    xr.a.re = shfl_down(sb.a.re, 1); xr.a.im = shfl_down(sb.a.im, 1);
    xr.g.re = shfl_down(sb.g.re, 1); xr.g.im = shfl_down(sb.g.im, 1);
    if (lane > 0) cf = cfma(xl.a, cf, xl.f);
    if (lane < kWave - 1) cb = cfma(xr.a, cb, xr.g);

    // Forward sweep: h+ at every point of the chunk.
    C<T> h = cf;
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      h = cfma(ex[j], h, C<T>{bb[j], T(0)});
      if (OUT & kOutVal) acc[j] = fma(om_re, h.re, fma(-om_im, h.im, acc[j]));
      if (OUT & kOutDer) dacc[j] = fma(dm_re, h.re, fma(-dm_im, h.im, dacc[j]));
    }
    // Backward sweep: h- (exclusive) at every point.
    C<T> g = cb;
#pragma unroll
    for (int j = kScanChunk - 1; j >= 0; --j) {
      if (OUT & kOutVal) acc[j] = fma(om_re, g.re, fma(-om_im, g.im, acc[j]));
      if (OUT & kOutDer) dacc[j] = fma(-dm_re, g.re, fma(dm_im, g.im, dacc[j]));
      g = cmul(ex[j], cadd(g, C<T>{bb[j], T(0)}));
    }
  }

  uint32_t myid[kScanChunk];
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) myid[j] = st.id[lds_pos(e0 + j)];
  scatter_chunk<T, OUT>(out, myid, acc, dacc);
}

// ---------------------------------------------------------------------------
// k_final_fast: tiles short on the decay scale (moment count K known from
// k_reduce).  The carry into each thread's chunk comes from the other chunks'
// power moments about the tile centre c:
//   h+ before the chunk  = E_f (CF eG + sum_m tau^m P_m / m!),    E_f = exp(-tau (z_s - c)),
//   h- at its last point = E_b (CB eF + sum_m (-tau)^m S_m / m!), E_b = exp(-tau (c - z_e)),
// with P_m / S_m the moments of the tile's points before / after the chunk,
// CF, CB the tile carries, eF = exp(-tau hf), eG = exp(-tau hg) (from k_reduce).
// The moments are mode-independent, so only two short Taylor series and two
// Horner sums per chunk and mode remain besides the sweeps.
// ---------------------------------------------------------------------------
template <class T>
union FastLds {
  Staged<T> st;
  struct {
    T pre[kFastMoments + 1][kScanThreads];   // moments of the tile's points before each chunk
    T suf[kFastMoments + 1][kScanThreads];   // ... and after it
  } mom;
};

template <class T, int NM, int OUT>
__global__ __launch_bounds__(kScanThreads) void k_final_fast(
    const void* keys0, const void* keys1, const PassInfo* __restrict__ pass,
    const T* __restrict__ bs, const uint32_t* __restrict__ ids, int64_t P, Modes md,
    const T* __restrict__ agg, const T* __restrict__ carry, const int32_t* __restrict__ tile_k,
    ScanOut<T> out) {
  const int64_t tile = blockIdx.x;
  const int K = tile_k[tile];
  if (K < 0 || K > kFastMoments) return;
  const KeyView<T> keys = key_view<T>(keys0, keys1, pass);
  __shared__ FastLds<T> lds;
  __shared__ T mtot[kFastMoments + 1][kScanWaves];
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int64_t t0 = tile * kScanTile;
  const int n = (int)((P - t0) < kScanTile ? (P - t0) : kScanTile);

  {
    // All of this thread's loads are issued before any is used; they are the
    // last reads of the sorted points in this call, so they are nontemporal.
    constexpr int R = kScanTile / kScanThreads;
    T zr[R], br[R];
    uint32_t sr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t p = t0 + tid + r * kScanThreads;
      const bool in = p < P;
      zr[r] = in ? __builtin_nontemporal_load(&keys.z[p]) : T(0);
      br[r] = in ? __builtin_nontemporal_load(&bs[p]) : T(0);
      sr[r] = in ? __builtin_nontemporal_load(&ids[p]) : kNoSlot;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = lds_pos(tid + r * kScanThreads);
      lds.st.z[q] = zr[r];
      lds.st.b[q] = br[r];
      lds.st.id[q] = sr[r];
    }
  }
  const T zfirst = keys(t0);
  const T zprev = t0 > 0 ? keys(t0 - 1) : zfirst;
  const T zlast = keys(t0 + n - 1);
  const T c = zprev + (zlast - zprev) * T(0.5);
  __syncthreads();

  // Chunk: gaps, strengths, offsets from the centre, ids, the point before
  // it (zs) and its last point (ze).
  const int e0 = tid * kScanChunk;
  T dz[kScanChunk], bb[kScanChunk], sc[kScanChunk];
  uint32_t myid[kScanChunk];
  T dzmax = T(0);
  T zl = tid == 0 ? zprev : (e0 - 1 < n ? lds.st.z[lds_pos(e0 - 1)] : zlast);
  const T zs = zl;
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    const int e = e0 + j;
    const bool valid = e < n;
    const T zj = lds.st.z[lds_pos(e)];
    dz[j] = valid ? zj - zl : T(0);
    bb[j] = lds.st.b[lds_pos(e)];
    sc[j] = valid ? zj - c : T(0);
    myid[j] = lds.st.id[lds_pos(e)];
    zl = valid ? zj : zl;
    dzmax = dz[j] > dzmax ? dz[j] : dzmax;
  }
  const T ze = zl;
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const T other = shfl_xor(dzmax, o);
    dzmax = other > dzmax ? other : dzmax;
  }
  __syncthreads();   // the staging area becomes the moment tables

  // Chunk moments nu_m = sum_j b_j (z_j - c)^m, their in-wave inclusive sums
  // (into pre) and the chunk's own values (into suf) for now.
  {
    T pw[kScanChunk];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) pw[j] = bb[j];
    for (int m = 0; m <= K; ++m) {
      T nu = T(0);
#pragma unroll
      for (int j = 0; j < kScanChunk; ++j) {
        nu += pw[j];
        pw[j] *= sc[j];
      }
      T inc = nu;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const T v = shfl_up(inc, o);
        if (lane >= o) inc += v;
      }
      if (lane == kWave - 1) mtot[m][wave] = inc;
      lds.mom.pre[m][tid] = inc;
      lds.mom.suf[m][tid] = nu;
    }
  }
  __syncthreads();
  for (int m = 0; m <= K; ++m) {
    T off = T(0), tot = T(0);
#pragma unroll
    for (int w = 0; w < kScanWaves; ++w) {
      const T v = mtot[m][w];
      if (w < wave) off += v;
      tot += v;
    }
    const T inc = lds.mom.pre[m][tid];
    const T nu = lds.mom.suf[m][tid];
    lds.mom.pre[m][tid] = off + (inc - nu);   // before the chunk
    lds.mom.suf[m][tid] = (tot - off) - inc;  // after the chunk
  }

  T acc[kScanChunk], dacc[kScanChunk];
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    acc[j] = T(0);
    dacc[j] = T(0);
  }
  const T xf = zs - c;
  const T xb = c - ze;

#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
    const T om_re = T(md.om_re[k]), om_im = T(md.om_im[k]);
    const T dm_re = T(md.dom_re[k]), dm_im = T(md.dom_im[k]);

    // Carries into the chunk.  exp(-tau xf), exp(-tau xb) with |tau x| <= r:
    // degree K suffices; sum_m tau^m P_m / m! and sum_m (-tau)^m S_m / m! by Horner.
    C<T> ef = {T(0), T(0)}, eb = {T(0), T(0)}, fs = {T(0), T(0)}, gs = {T(0), T(0)};
    for (int m = K; m >= 0; --m) {
      const T c_re = T(md.coef_re[k][m]), c_im = T(md.coef_im[k][m]);
      ef.re = fma(ef.re, xf, c_re);
      ef.im = fma(ef.im, xf, c_im);
      eb.re = fma(eb.re, xb, c_re);
      eb.im = fma(eb.im, xb, c_im);
      const T f = T(kInvFact.v[m]);
      fs = cfma(fs, C<T>{tr, ti}, C<T>{lds.mom.pre[m][tid] * f, T(0)});
      gs = cfma(gs, C<T>{-tr, -ti}, C<T>{lds.mom.suf[m][tid] * f, T(0)});
    }
    const T* ag = agg + ((size_t)tile * NM + k) * kAggStride;
    const T* cr = carry + ((size_t)tile * NM + k) * 4;
    const C<T> tf = cfma(C<T>{cr[0], cr[1]}, C<T>{ag[8], ag[9]}, fs);   // CF eG + fs
    const C<T> tb = cfma(C<T>{cr[2], cr[3]}, C<T>{ag[6], ag[7]}, gs);   // CB eF + gs

    // Mode exponentials of the chunk's gaps.
    const double rr = md.tau_abs[k] * (double)dzmax;
    int D = kTaylorMax;
#pragma unroll
    for (int d = kTaylorMax; d >= 1; --d)
      if (rr <= md.taylor_thr[d]) D = d;
    const T dz_lim = T(md.dz_lim[k]);
    C<T> ex[kScanChunk];
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
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j)
      if (dz[j] > dz_lim) ex[j] = exp_neg_general<T>(tr, ti, dz[j]);

    C<T> h = cmul(ef, tf);
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      h = cfma(ex[j], h, C<T>{bb[j], T(0)});
      if (OUT & kOutVal) acc[j] = fma(om_re, h.re, fma(-om_im, h.im, acc[j]));
      if (OUT & kOutDer) dacc[j] = fma(dm_re, h.re, fma(-dm_im, h.im, dacc[j]));
    }
    C<T> g = cmul(eb, tb);
#pragma unroll
    for (int j = kScanChunk - 1; j >= 0; --j) {
      if (OUT & kOutVal) acc[j] = fma(om_re, g.re, fma(-om_im, g.im, acc[j]));
      if (OUT & kOutDer) dacc[j] = fma(-dm_re, g.re, fma(dm_im, g.im, dacc[j]));
      g = cmul(ex[j], cadd(g, C<T>{bb[j], T(0)}));
    }
  }

  scatter_chunk<T, OUT>(out, myid, acc, dacc);
}

template <class T>
__global__ void k_fill_zero(T* __restrict__ u, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) u[i] = T(0);
}

template <class T>
hipError_t carry_tiles(const Workspace& w, int nq, hipStream_t s) {
  return launch_carries<T>(AggMaps<T>{(const T*)w.agg, nq}, w.scan_tiles, nq, (T*)w.chunk_agg,
                           (T*)w.chunk_carry, (T*)w.carry, s);
}

template <class T, int NM, int OUT>
hipError_t scan_nm(const Workspace& w, const Modes& md, int64_t P, const T* b,
                   const ScanOut<T>& out, hipStream_t s, Timeline* tl) {
  const dim3 grid((unsigned)w.scan_tiles);
  hipLaunchKernelGGL((k_reduce<T, NM>), grid, dim3(kWave), 0, s, w.keys[0], w.keys[1], w.pass, b,
                     P, md, (T*)w.agg, w.tile_k);
  tl->mark(s);
  (void)carry_tiles<T>(w, NM, s);
  tl->mark(s);
  hipLaunchKernelGGL((k_final_fast<T, NM, OUT>), grid, dim3(kScanThreads), 0, s, w.keys[0],
                     w.keys[1], w.pass, b, w.ids, P, md, (const T*)w.agg, (const T*)w.carry,
                     w.tile_k, out);
  hipLaunchKernelGGL((k_final<T, NM, OUT>), grid, dim3(kScanThreads), 0, s, w.keys[0], w.keys[1],
                     w.pass, b, w.ids, P, md, (const T*)w.carry, w.tile_k, out);
  tl->mark(s);
  return hipGetLastError();
}

template <class T, int NM>
hipError_t scan_out(const Workspace& w, const Modes& md, int64_t P, const T* b,
                    const ScanOut<T>& out, hipStream_t s, Timeline* tl) {
  const int kind = (out.val ? kOutVal : 0) | (out.der ? kOutDer : 0);
  switch (kind) {
    case kOutVal: return scan_nm<T, NM, kOutVal>(w, md, P, b, out, s, tl);
    case kOutVal | kOutDer: return scan_nm<T, NM, kOutVal | kOutDer>(w, md, P, b, out, s, tl);
    default: return hipErrorInvalidValue;   // the adjoint has its own kernels
  }
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
hipError_t scan_points(const Workspace& w, const Modes& md, int64_t P, const T* b,
                       const ScanOut<T>& out, hipStream_t s, Timeline* tl) {
  switch (md.n) {
    case 1: return scan_out<T, 1>(w, md, P, b, out, s, tl);
    case 2: return scan_out<T, 2>(w, md, P, b, out, s, tl);
    case 3: return scan_out<T, 3>(w, md, P, b, out, s, tl);
    case 4: return scan_out<T, 4>(w, md, P, b, out, s, tl);
    case 5: return scan_out<T, 5>(w, md, P, b, out, s, tl);
    case 6: return scan_out<T, 6>(w, md, P, b, out, s, tl);
    case 7: return scan_out<T, 7>(w, md, P, b, out, s, tl);
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
                                        const ScanOut<double>&, hipStream_t, Timeline*);
template hipError_t scan_points<float>(const Workspace&, const Modes&, int64_t, const float*,
                                       const ScanOut<float>&, hipStream_t, Timeline*);
template hipError_t gather_strengths<double>(const Workspace&, int64_t, uint32_t, uint32_t,
                                             const double*, double*, hipStream_t);
template hipError_t gather_strengths<float>(const Workspace&, int64_t, uint32_t, uint32_t,
                                            const float*, float*, hipStream_t);
template hipError_t fill_zero<double>(double*, int64_t, hipStream_t);
template hipError_t fill_zero<float>(float*, int64_t, hipStream_t);

}  // namespace fgt
