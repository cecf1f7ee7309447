// Adjoint of the transform (the gradients of L = sum_i g_i u_i) on gfx950, as
// ONE pass over the sorted points that the forward transform left behind.
//
// Two strength channels share every mode exponential e_p = exp(-tau (z_p - z_{p-1})):
//   channel 0: b_p = alpha_j at the sources (the forward strengths); its sweeps
//              give, at each target i, the x-derivative of the transform
//              u'_i = sum_k Re(-tau_k omega_k (h+ - h-)), so dL/dx_i = g_i u'_i;
//   channel 1: b_p = g_i at the targets (the transposed transform, sources and
//              targets swapped, the Gaussian being even); its sweeps give, at each
//              source j, v_j = sum_k Re(omega_k (h+ + h-)) = dL/dalpha_j and
//              v'_j, with dL/dy_j = alpha_j v'_j.
// h+ holds the sources to the left of a point (sign +1 of the derivative), h-
// those to its right (sign -1), as in (4.4).  The scaling identity
// u(c x, c y; c^2 delta) = u(x, y; delta), exact for the SOE since its nodes
// scale as 1/sqrt(delta), gives
//   dL/ddelta = -(sum_i (x_i - c) dL/dx_i + sum_j (y_j - c) dL/dy_j) / (2 delta)
// for any c (translation invariance); each tile adds its part, about the
// midpoint c of the sorted coordinates.
//
// Kernels (the reduce-then-scan of the forward, with 2 x modes scans):
//   k_adj_reduce      one wave per tile: gathers g into sorted order once, then
//                     the tile maps (A, F, G) of both channels (power moments of
//                     the strengths when the tile is short on the decay scale)
//   carries           the three-level tile carries over 2 x modes scans
//   k_adj_final_fast  tiles with at most kAdjMoments moments: chunk carries from
//                     the moments, both channels' sweeps, scatter of the gradients;
//                     the other tiles (wide, or more moments) by chunk and wave
//                     scans of both channels, in the same launch
//   k_adj_delta       sum of the tiles' parts of dL/ddelta
#include "fgt_device.h"

namespace fgt {
namespace {

constexpr int kAdjMoments = 8;

__device__ __forceinline__ int lds_pos(int e) { return e + e / kScanChunk; }

// ---------------------------------------------------------------------------
// k_adj_reduce
// ---------------------------------------------------------------------------
template <class T, int NM>
__global__ __launch_bounds__(kWave) void k_adj_reduce(const void* keys0, const void* keys1,
                                                      const PassInfo* __restrict__ pass,
                                                      const T* __restrict__ b,
                                                      const uint32_t* __restrict__ ids,
                                                      const T* __restrict__ g, int64_t N,
                                                      int64_t P, Modes md, T* __restrict__ bt,
                                                      T* __restrict__ agg,
                                                      int32_t* __restrict__ tile_k) {
  constexpr int NQ = 2 * NM;
  const KeyView<T> keys = key_view<T>(keys0, keys1, pass);
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t t0 = tile * kScanTile;
  const int n = (int)((P - t0) < kScanTile ? (P - t0) : kScanTile);
  const uint32_t M = (uint32_t)(P - N);
  const T zfirst = keys(t0);
  const T zprev = t0 > 0 ? keys(t0 - 1) : zfirst;
  const T zlast = keys(t0 + n - 1);
  const T c = zprev + (zlast - zprev) * T(0.5);
  const T hf = zlast - c;
  const T hg = c - zprev;
  const T span = zlast - zprev;
  const T r = T(md.tau_abs_max) * (hf > hg ? hf : hg);
  int K = 0;
  {
    const T er = exp_t(r);
    T t = r;
    while (t * er > T(Prec<T>::kUnit) && K < kMomentMax) {
      ++K;
      t *= r / T(K + 1);
    }
    if (t * er > T(Prec<T>::kUnit)) K = -1;
  }
  if (lane == 0) tile_k[tile] = K;

  // Channel 1 strengths in sorted order: g_i at target i, 0 at a source.
  auto gather = [&](int e) -> T {
    const uint32_t o = ids[t0 + e] - (uint32_t)N;
    return o < M ? g[o] : T(0);
  };

  if (K >= 0) {
    T mu0[kMomentMax + 1], mu1[kMomentMax + 1];
#pragma unroll
    for (int m = 0; m <= kMomentMax; ++m) {
      mu0[m] = T(0);
      mu1[m] = T(0);
    }
    for (int e = lane; e < n; e += kWave) {
      const T s = keys(t0 + e) - c;
      const T wt = gather(e);
      bt[t0 + e] = wt;
      T p0 = b[t0 + e], p1 = wt;
      mu0[0] += p0;
      mu1[0] += p1;
#pragma unroll
      for (int m = 1; m <= kMomentMax; ++m) {
        if (m <= K) {
          p0 *= s;
          p1 *= s;
          mu0[m] += p0;
          mu1[m] += p1;
        }
      }
    }
#pragma unroll
    for (int m = 0; m <= kMomentMax; ++m) {
      if (m <= K) {
#pragma unroll
        for (int o = kWave / 2; o >= 1; o >>= 1) {
          mu0[m] += shfl_xor(mu0[m], o);
          mu1[m] += shfl_xor(mu1[m], o);
        }
      }
    }
    if (lane < NQ) {
      const int ch = lane / NM;
      const int k = lane % NM;
      const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
      T top = T(0);
#pragma unroll
      for (int m = 0; m <= kMomentMax; ++m)
        if (m == K) top = ch ? mu1[m] : mu0[m];
      C<T> fs = {top * T(kInvFact.v[K]), T(0)};
      C<T> gs = fs;
#pragma unroll
      for (int m = kMomentMax - 1; m >= 0; --m) {
        if (m < K) {
          const C<T> cm = {(ch ? mu1[m] : mu0[m]) * T(kInvFact.v[m]), T(0)};
          fs = cfma(fs, C<T>{tr, ti}, cm);
          gs = cfma(gs, C<T>{-tr, -ti}, cm);
        }
      }
      const C<T> ef = exp_neg_general<T>(tr, ti, hf);
      const C<T> eg = exp_neg_general<T>(tr, ti, hg);
      const C<T> a = exp_neg_general<T>(tr, ti, span);
      const C<T> f = cmul(ef, fs);
      const C<T> gg = cmul(eg, gs);
      T* o = agg + ((size_t)tile * NQ + lane) * kAggStride;
      o[0] = a.re; o[1] = a.im;
      o[2] = f.re; o[3] = f.im;
      o[4] = gg.re; o[5] = gg.im;
      o[6] = ef.re; o[7] = ef.im;
      o[8] = eg.re; o[9] = eg.im;
    }
    return;
  }

  // Wide tile: each lane folds both channels over kPer consecutive points.
  constexpr int kPer = kScanTile / kWave;
  for (int e = lane; e < n; e += kWave) bt[t0 + e] = gather(e);
  const int e0 = lane * kPer;
  const int cnt = n - e0 < 0 ? 0 : (n - e0 < kPer ? n - e0 : kPer);
#pragma unroll 1
  for (int q = 0; q < NQ; ++q) {
    const int ch = q / NM;
    const int k = q % NM;
    const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
    Seg<T> s = seg_identity<T>();
    T zl = e0 == 0 ? zprev : (cnt > 0 ? keys(t0 + e0 - 1) : zlast);
    for (int j = 0; j < cnt; ++j) {
      const T zj = keys(t0 + e0 + j);
      const C<T> ex = exp_neg_general<T>(tr, ti, zj - zl);
      const T w = ch ? gather(e0 + j) : b[t0 + e0 + j];
      s.a = cmul(s.a, ex);
      s.f = cfma(ex, s.f, C<T>{w, T(0)});
      zl = zj;
    }
    C<T> gg = {T(0), T(0)};
    for (int j = cnt - 1; j >= 0; --j) {
      const T zj = keys(t0 + e0 + j);
      const T zb = (e0 + j == 0) ? zprev : keys(t0 + e0 + j - 1);
      const C<T> ex = exp_neg_general<T>(tr, ti, zj - zb);
      const T w = ch ? gather(e0 + j) : b[t0 + e0 + j];
      gg = cmul(ex, cadd(gg, C<T>{w, T(0)}));
    }
    s.g = gg;
    Seg<T> pf, sb;
    wave_scans(s, lane, pf, sb);
    T* o = agg + ((size_t)tile * NQ + q) * kAggStride;
    if (lane == kWave - 1) {
      o[0] = pf.a.re; o[1] = pf.a.im;
      o[2] = pf.f.re; o[3] = pf.f.im;
    }
    if (lane == 0) {
      o[4] = sb.g.re; o[5] = sb.g.im;
    }
  }
}

// Outputs of the adjoint scan.
template <class T>
struct AdjOut {
  T* dx;          // [M] or null
  T* dalpha;      // [N] or null
  T* dy;          // [N] or null
  double* part;   // [tiles] parts of sum (z - c) * grad, or null
  int64_t N, M;
};

// Scatter of one chunk and its part of the delta-gradient sum (about zc).
template <class T>
__device__ __forceinline__ double adj_scatter(const AdjOut<T>& out, const uint32_t* myid,
                                              const T* bb, const T* bg, const T* za,
                                              const T* dacc0, const T* acc1, const T* dacc1,
                                              double zc) {
  double part = 0.0;
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    const uint32_t id = myid[j];
    if (id == kNoSlot) continue;
    if ((int64_t)id >= out.N) {
      const uint32_t o = id - (uint32_t)out.N;
      if (o < (uint32_t)out.M) {
        const T v = bg[j] * dacc0[j];
        if (out.dx) out.dx[o] = v;
        part += ((double)za[j] - zc) * (double)v;
      }
    } else {
      const T v = bb[j] * dacc1[j];
      if (out.dalpha) out.dalpha[id] = acc1[j];
      if (out.dy) out.dy[id] = v;
      part += ((double)za[j] - zc) * (double)v;
    }
  }
  return part;
}

template <class T>
__device__ __forceinline__ void block_part(double part, double* __restrict__ dst, double* wsum) {
  for (int o = kWave / 2; o >= 1; o >>= 1) part += __shfl_xor(part, o, kWave);
  if (threadIdx.x % kWave == 0) wsum[threadIdx.x / kWave] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kScanWaves; ++w) s += wsum[w];
    *dst = s;
  }
}

template <class T>
struct Staged2 {
  T z[kScanTile + kScanTile / kScanChunk];
  T b[kScanTile + kScanTile / kScanChunk];
  T bt[kScanTile + kScanTile / kScanChunk];
  uint32_t id[kScanTile + kScanTile / kScanChunk];
};

template <class T>
union AdjFastLds {
  Staged2<T> st;
  struct {
    T pre[2][kAdjMoments + 1][kScanThreads];
    T suf[2][kAdjMoments + 1][kScanThreads];
  } mom;
};

// Loads this thread's share of the tile into LDS (coalesced), all loads first.
// These are the last reads of the sorted arrays in the call, so they are
// nontemporal: they leave the caches to the scattered gradient writes.
template <class T>
__device__ __forceinline__ void stage_tile(Staged2<T>& st, const KeyView<T>& keys, const T* b,
                                           const T* bt, const uint32_t* ids, int64_t t0,
                                           int64_t P) {
  constexpr int R = kScanTile / kScanThreads;
  const int tid = threadIdx.x;
  T zr[R], br[R], gr[R];
  uint32_t ir[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t p = t0 + tid + r * kScanThreads;
    const bool in = p < P;
    zr[r] = in ? __builtin_nontemporal_load(&keys.z[p]) : T(0);
    br[r] = in ? __builtin_nontemporal_load(&b[p]) : T(0);
    gr[r] = in ? __builtin_nontemporal_load(&bt[p]) : T(0);
    ir[r] = in ? __builtin_nontemporal_load(&ids[p]) : kNoSlot;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = lds_pos(tid + r * kScanThreads);
    st.z[q] = zr[r];
    st.b[q] = br[r];
    st.bt[q] = gr[r];
    st.id[q] = ir[r];
  }
}

// ---------------------------------------------------------------------------
// Tiles outside the moment path (wide, or many moments): chunk and wave scans
// of both channels.  Run by k_adj_final_fast's block for such a tile, in the
// staging part of its LDS.
// ---------------------------------------------------------------------------
template <class T, int NM>
__device__ __forceinline__ void adj_general_tile(
    Staged2<T>& st, Seg<T> (&wtot)[2][kScanWaves][2], double* wsum, const KeyView<T>& keys,
    const T* __restrict__ b, const T* __restrict__ bt, const uint32_t* __restrict__ ids,
    int64_t P, const Modes& md, const T* __restrict__ carry, const AdjOut<T>& out, int64_t tile) {
  constexpr int NQ = 2 * NM;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int64_t t0 = tile * kScanTile;
  const int n = (int)((P - t0) < kScanTile ? (P - t0) : kScanTile);

  stage_tile(st, keys, b, bt, ids, t0, P);
  T zprev = t0 > 0 ? keys(t0 - 1) : T(0);
  const double zc = 0.5 * ((double)keys(0) + (double)keys(P - 1));
  __syncthreads();

  const int e0 = tid * kScanChunk;
  T dz[kScanChunk], bb[kScanChunk], bg[kScanChunk], za[kScanChunk];
  uint32_t myid[kScanChunk];
  T dzmax = T(0);
  {
    T zl = tid == 0 ? (t0 > 0 ? zprev : st.z[lds_pos(0)]) : st.z[lds_pos(e0 - 1)];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      const int e = e0 + j;
      const T zj = st.z[lds_pos(e)];
      dz[j] = (e < n) ? zj - zl : T(0);
      bb[j] = st.b[lds_pos(e)];
      bg[j] = st.bt[lds_pos(e)];
      za[j] = zj;
      myid[j] = st.id[lds_pos(e)];
      zl = (e < n) ? zj : zl;
      dzmax = dz[j] > dzmax ? dz[j] : dzmax;
    }
  }
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const T other = shfl_xor(dzmax, o);
    dzmax = other > dzmax ? other : dzmax;
  }

  T dacc0[kScanChunk], acc1[kScanChunk], dacc1[kScanChunk];
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    dacc0[j] = T(0);
    acc1[j] = T(0);
    dacc1[j] = T(0);
  }

#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
    const T om_re = T(md.om_re[k]), om_im = T(md.om_im[k]);
    const T dm_re = T(md.dom_re[k]), dm_im = T(md.dom_im[k]);
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

    C<T> cf[2], cb[2];
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      T w[kScanChunk];
#pragma unroll
      for (int j = 0; j < kScanChunk; ++j) w[j] = ch ? bg[j] : bb[j];
      Seg<T> s;
      s.a = ex[0];
      s.f = {w[0], T(0)};
#pragma unroll
      for (int j = 1; j < kScanChunk; ++j) {
        s.a = cmul(s.a, ex[j]);
        s.f = cfma(ex[j], s.f, C<T>{w[j], T(0)});
      }
      s.g = {T(0), T(0)};
#pragma unroll
      for (int j = kScanChunk - 1; j >= 0; --j) s.g = cmul(ex[j], cadd(s.g, C<T>{w[j], T(0)}));
      Seg<T> pf, sb;
      wave_scans(s, lane, pf, sb);
      if (lane == kWave - 1) wtot[ch][wave][0] = pf;
      if (lane == 0) wtot[ch][wave][1] = sb;
      __syncthreads();
      const T* cr = carry + ((size_t)tile * NQ + ch * NM + k) * 4;
      C<T> f = {cr[0], cr[1]};
      C<T> g = {cr[2], cr[3]};
      for (int ww = 0; ww < wave; ++ww) f = cfma(wtot[ch][ww][0].a, f, wtot[ch][ww][0].f);
      for (int ww = kScanWaves - 1; ww > wave; --ww) g = cfma(wtot[ch][ww][1].a, g, wtot[ch][ww][1].g);
      Seg<T> xl, xr;
      xl.a.re = shfl_up(pf.a.re, 1); xl.a.im = shfl_up(pf.a.im, 1);
      xl.f.re = shfl_up(pf.f.re, 1); xl.f.im = shfl_up(pf.f.im, 1);
      xr.a.re = shfl_down(sb.a.re, 1); xr.a.im = shfl_down(sb.a.im, 1);
      xr.g.re = shfl_down(sb.g.re, 1); xr.g.im = shfl_down(sb.g.im, 1);
      if (lane > 0) f = cfma(xl.a, f, xl.f);
      if (lane < kWave - 1) g = cfma(xr.a, g, xr.g);
      cf[ch] = f;
      cb[ch] = g;
      __syncthreads();   // wtot of this channel is read before it is rewritten
    }

    C<T> h0 = cf[0], h1 = cf[1];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      h0 = cfma(ex[j], h0, C<T>{bb[j], T(0)});
      h1 = cfma(ex[j], h1, C<T>{bg[j], T(0)});
      dacc0[j] = fma(dm_re, h0.re, fma(-dm_im, h0.im, dacc0[j]));
      acc1[j] = fma(om_re, h1.re, fma(-om_im, h1.im, acc1[j]));
      dacc1[j] = fma(dm_re, h1.re, fma(-dm_im, h1.im, dacc1[j]));
    }
    C<T> g0 = cb[0], g1 = cb[1];
#pragma unroll
    for (int j = kScanChunk - 1; j >= 0; --j) {
      dacc0[j] = fma(-dm_re, g0.re, fma(dm_im, g0.im, dacc0[j]));
      acc1[j] = fma(om_re, g1.re, fma(-om_im, g1.im, acc1[j]));
      dacc1[j] = fma(-dm_re, g1.re, fma(dm_im, g1.im, dacc1[j]));
      g0 = cmul(ex[j], cadd(g0, C<T>{bb[j], T(0)}));
      g1 = cmul(ex[j], cadd(g1, C<T>{bg[j], T(0)}));
    }
  }

  const double part = adj_scatter(out, myid, bb, bg, za, dacc0, acc1, dacc1, zc);
  if (out.part) block_part<T>(part, out.part + tile, wsum);
}

// ---------------------------------------------------------------------------
// k_adj_final_fast
// ---------------------------------------------------------------------------
template <class T, int NM>
__global__ __launch_bounds__(kScanThreads) void k_adj_final_fast(
    const void* keys0, const void* keys1, const PassInfo* __restrict__ pass,
    const T* __restrict__ b, const T* __restrict__ bt, const uint32_t* __restrict__ ids,
    int64_t P, Modes md, const T* __restrict__ agg, const T* __restrict__ carry,
    const int32_t* __restrict__ tile_k, AdjOut<T> out) {
  constexpr int NQ = 2 * NM;
  const int64_t tile = blockIdx.x;
  const int K = tile_k[tile];
  const KeyView<T> keys = key_view<T>(keys0, keys1, pass);
  __shared__ AdjFastLds<T> lds;
  __shared__ T mtot[2][kAdjMoments + 1][kScanWaves];
  __shared__ double wsum[kScanWaves];
  if (K < 0 || K > kAdjMoments) {
    __shared__ Seg<T> wtot[2][kScanWaves][2];   // per channel and wave: forward, backward totals
    adj_general_tile<T, NM>(lds.st, wtot, wsum, keys, b, bt, ids, P, md, carry, out, tile);
    return;
  }
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int64_t t0 = tile * kScanTile;
  const int n = (int)((P - t0) < kScanTile ? (P - t0) : kScanTile);

  stage_tile(lds.st, keys, b, bt, ids, t0, P);
  const T zfirst = keys(t0);
  const T zprev = t0 > 0 ? keys(t0 - 1) : zfirst;
  const T zlast = keys(t0 + n - 1);
  const T c = zprev + (zlast - zprev) * T(0.5);
  const double zc = 0.5 * ((double)keys(0) + (double)keys(P - 1));
  __syncthreads();

  const int e0 = tid * kScanChunk;
  T dz[kScanChunk], bb[kScanChunk], bg[kScanChunk], sc[kScanChunk], za[kScanChunk];
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
    bg[j] = lds.st.bt[lds_pos(e)];
    sc[j] = valid ? zj - c : T(0);
    za[j] = zj;
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

  // Moments of both channels: in-wave inclusive sums into pre, own values into suf.
  {
    T p0[kScanChunk], p1[kScanChunk];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      p0[j] = bb[j];
      p1[j] = bg[j];
    }
    for (int m = 0; m <= K; ++m) {
      T nu0 = T(0), nu1 = T(0);
#pragma unroll
      for (int j = 0; j < kScanChunk; ++j) {
        nu0 += p0[j];
        nu1 += p1[j];
        p0[j] *= sc[j];
        p1[j] *= sc[j];
      }
      T i0 = nu0, i1 = nu1;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const T v0 = shfl_up(i0, o);
        const T v1 = shfl_up(i1, o);
        if (lane >= o) {
          i0 += v0;
          i1 += v1;
        }
      }
      if (lane == kWave - 1) {
        mtot[0][m][wave] = i0;
        mtot[1][m][wave] = i1;
      }
      lds.mom.pre[0][m][tid] = i0;
      lds.mom.pre[1][m][tid] = i1;
      lds.mom.suf[0][m][tid] = nu0;
      lds.mom.suf[1][m][tid] = nu1;
    }
  }
  __syncthreads();
  for (int ch = 0; ch < 2; ++ch) {
    for (int m = 0; m <= K; ++m) {
      T off = T(0), tot = T(0);
#pragma unroll
      for (int w = 0; w < kScanWaves; ++w) {
        const T v = mtot[ch][m][w];
        if (w < wave) off += v;
        tot += v;
      }
      const T inc = lds.mom.pre[ch][m][tid];
      const T nu = lds.mom.suf[ch][m][tid];
      lds.mom.pre[ch][m][tid] = off + (inc - nu);
      lds.mom.suf[ch][m][tid] = (tot - off) - inc;
    }
  }

  T dacc0[kScanChunk], acc1[kScanChunk], dacc1[kScanChunk];
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) {
    dacc0[j] = T(0);
    acc1[j] = T(0);
    dacc1[j] = T(0);
  }
  const T xf = zs - c;
  const T xb = c - ze;

#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    const T tr = T(md.tau_re[k]), ti = T(md.tau_im[k]);
    const T om_re = T(md.om_re[k]), om_im = T(md.om_im[k]);
    const T dm_re = T(md.dom_re[k]), dm_im = T(md.dom_im[k]);

    C<T> ef = {T(0), T(0)}, eb = {T(0), T(0)};
    C<T> fs0 = {T(0), T(0)}, gs0 = {T(0), T(0)}, fs1 = {T(0), T(0)}, gs1 = {T(0), T(0)};
    for (int m = K; m >= 0; --m) {
      const T c_re = T(md.coef_re[k][m]), c_im = T(md.coef_im[k][m]);
      ef.re = fma(ef.re, xf, c_re);
      ef.im = fma(ef.im, xf, c_im);
      eb.re = fma(eb.re, xb, c_re);
      eb.im = fma(eb.im, xb, c_im);
      const T f = T(kInvFact.v[m]);
      fs0 = cfma(fs0, C<T>{tr, ti}, C<T>{lds.mom.pre[0][m][tid] * f, T(0)});
      gs0 = cfma(gs0, C<T>{-tr, -ti}, C<T>{lds.mom.suf[0][m][tid] * f, T(0)});
      fs1 = cfma(fs1, C<T>{tr, ti}, C<T>{lds.mom.pre[1][m][tid] * f, T(0)});
      gs1 = cfma(gs1, C<T>{-tr, -ti}, C<T>{lds.mom.suf[1][m][tid] * f, T(0)});
    }
    const T* ag = agg + ((size_t)tile * NQ + k) * kAggStride;
    const T* c0 = carry + ((size_t)tile * NQ + k) * 4;
    const T* c1 = carry + ((size_t)tile * NQ + NM + k) * 4;
    const C<T> eG = {ag[8], ag[9]}, eF = {ag[6], ag[7]};
    const C<T> tf0 = cfma(C<T>{c0[0], c0[1]}, eG, fs0);
    const C<T> tb0 = cfma(C<T>{c0[2], c0[3]}, eF, gs0);
    const C<T> tf1 = cfma(C<T>{c1[0], c1[1]}, eG, fs1);
    const C<T> tb1 = cfma(C<T>{c1[2], c1[3]}, eF, gs1);

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

    C<T> h0 = cmul(ef, tf0), h1 = cmul(ef, tf1);
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      h0 = cfma(ex[j], h0, C<T>{bb[j], T(0)});
      h1 = cfma(ex[j], h1, C<T>{bg[j], T(0)});
      dacc0[j] = fma(dm_re, h0.re, fma(-dm_im, h0.im, dacc0[j]));
      acc1[j] = fma(om_re, h1.re, fma(-om_im, h1.im, acc1[j]));
      dacc1[j] = fma(dm_re, h1.re, fma(-dm_im, h1.im, dacc1[j]));
    }
    C<T> g0 = cmul(eb, tb0), g1 = cmul(eb, tb1);
#pragma unroll
    for (int j = kScanChunk - 1; j >= 0; --j) {
      dacc0[j] = fma(-dm_re, g0.re, fma(dm_im, g0.im, dacc0[j]));
      acc1[j] = fma(om_re, g1.re, fma(-om_im, g1.im, acc1[j]));
      dacc1[j] = fma(-dm_re, g1.re, fma(dm_im, g1.im, dacc1[j]));
      g0 = cmul(ex[j], cadd(g0, C<T>{bb[j], T(0)}));
      g1 = cmul(ex[j], cadd(g1, C<T>{bg[j], T(0)}));
    }
  }

  const double part = adj_scatter(out, myid, bb, bg, za, dacc0, acc1, dacc1, zc);
  if (out.part) block_part<T>(part, out.part + tile, wsum);
}

template <class T>
__global__ __launch_bounds__(256) void k_adj_delta(const double* __restrict__ part, int64_t n,
                                                   double scale, T* __restrict__ out) {
  __shared__ double wsum[4];
  // Eight partial sums a thread, so that eight loads are in flight (a fixed
  // order: the result is the same on every run).
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t i = threadIdx.x;
  for (; i + 7 * 256 < n; i += 8 * 256) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] += part[i + q * 256];
  }
  for (; i < n; i += 256) a[0] += part[i];
  double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  for (int o = kWave / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (threadIdx.x % kWave == 0) wsum[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (T)(scale * (wsum[0] + wsum[1] + wsum[2] + wsum[3]));
}

template <class T, int NM>
hipError_t adjoint_nm(const Workspace& w, const Modes& md, int64_t M, int64_t N, const T* g,
                      T* dx, T* dalpha, T* dy, T* ddelta, double delta, hipStream_t s) {
  const int64_t P = M + N;
  const dim3 grid((unsigned)w.scan_tiles);
  hipLaunchKernelGGL((k_adj_reduce<T, NM>), grid, dim3(kWave), 0, s, w.keys[0], w.keys[1], w.pass,
                     (const T*)w.b, (const uint32_t*)w.ids, g, N, P, md, (T*)w.bt, (T*)w.agg,
                     w.tile_k);
  const int nq = 2 * NM;
  hipError_t e = launch_carries<T>(AggMaps<T>{(const T*)w.agg, nq}, w.scan_tiles, nq,
                                   (T*)w.chunk_agg, (T*)w.chunk_carry, (T*)w.carry, s);
  if (e != hipSuccess) return e;
  const AdjOut<T> out{dx, dalpha, dy, ddelta ? w.tile_part : nullptr, N, M};
  hipLaunchKernelGGL((k_adj_final_fast<T, NM>), grid, dim3(kScanThreads), 0, s, w.keys[0],
                     w.keys[1], w.pass, (const T*)w.b, (const T*)w.bt, (const uint32_t*)w.ids, P,
                     md, (const T*)w.agg, (const T*)w.carry, w.tile_k, out);
  if (ddelta)
    hipLaunchKernelGGL(k_adj_delta<T>, dim3(1), dim3(256), 0, s, (const double*)w.tile_part,
                       w.scan_tiles, -0.5 / delta, ddelta);
  return hipGetLastError();
}

}  // namespace

template <class T>
hipError_t adjoint_points(const Workspace& w, const Modes& md, int64_t M, int64_t N, const T* g,
                          T* dx, T* dalpha, T* dy, T* ddelta, double delta, hipStream_t s) {
  switch (md.n) {
    case 1: return adjoint_nm<T, 1>(w, md, M, N, g, dx, dalpha, dy, ddelta, delta, s);
    case 2: return adjoint_nm<T, 2>(w, md, M, N, g, dx, dalpha, dy, ddelta, delta, s);
    case 3: return adjoint_nm<T, 3>(w, md, M, N, g, dx, dalpha, dy, ddelta, delta, s);
    case 4: return adjoint_nm<T, 4>(w, md, M, N, g, dx, dalpha, dy, ddelta, delta, s);
    case 5: return adjoint_nm<T, 5>(w, md, M, N, g, dx, dalpha, dy, ddelta, delta, s);
    case 6: return adjoint_nm<T, 6>(w, md, M, N, g, dx, dalpha, dy, ddelta, delta, s);
    case 7: return adjoint_nm<T, 7>(w, md, M, N, g, dx, dalpha, dy, ddelta, delta, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t adjoint_points<double>(const Workspace&, const Modes&, int64_t, int64_t,
                                           const double*, double*, double*, double*, double*,
                                           double, hipStream_t);
template hipError_t adjoint_points<float>(const Workspace&, const Modes&, int64_t, int64_t,
                                          const float*, float*, float*, float*, float*, double,
                                          hipStream_t);

}  // namespace fgt
