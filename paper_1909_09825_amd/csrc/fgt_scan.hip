// The SOE recurrences of Section 4 as parallel affine scans on gfx950.
//
// After the sort, point p of the merged sequence has coordinate z_p,
// strength b_p (alpha_j for source j, 0 for a target) and, for a target, its
// output slot.  For mode k (tau = tau0_k / sqrt(delta)) let
//     e_p = exp(-tau (z_p - z_{p-1})),   |e_p| <= 1 since z is sorted.
// The forward recurrence (4.5) over the merged sequence is
//     h+_p = e_p h+_{p-1} + b_p          (inclusive: sources at z_p count, (4.4))
// and the backward recurrence (4.6), exclusive of the point itself, is
//     h-_{p-1} = e_p (h-_p + b_p).
// One factor e_p serves both.  At a target u_p = sum_k Re(omega_k (h+_p + h-_p)), (4.1).
//
// A segment [s, e) of the sequence acts on the two recurrences as
//     h+_{e-1} = A h+_{s-1} + F,          h-_{s-1} = A h-_{e-1} + G,
//     A = prod_{p in seg} e_p,  F = sum b_q e^{-tau (z_{e-1} - z_q)},  G = sum b_q e^{-tau (z_q - z_{s-1})},
// and segments compose associatively:  (A1,F1,G1).(A2,F2,G2) = (A1 A2, A2 F1 + F2, G1 + A1 G2).
//
// Three kernels, reduce-then-scan over tiles of kScanTile points:
//   k_tiles<.., false>  per tile and mode: (A, F, G) of the tile       (reduce)
//   k_carry             per mode: exclusive prefix of F and suffix of G over tiles
//   k_tiles<.., true>   per tile: chunk -> wave -> tile scans, both sweeps with
//                       the carries, mode reduction, scatter u[slot] = value
// Inside a tile each thread owns kScanChunk consecutive points and runs the
// recurrences sequentially; chunks are combined with wave shuffles and LDS.
#include "fgt_internal.h"

namespace fgt {
namespace {

template <class T>
struct C {
  T re, im;
};

template <class T>
__device__ __forceinline__ C<T> cmul(C<T> a, C<T> b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// a * b + c
template <class T>
__device__ __forceinline__ C<T> cfma(C<T> a, C<T> b, C<T> c) {
  return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
template <class T>
__device__ __forceinline__ C<T> cadd(C<T> a, C<T> b) {
  return {a.re + b.re, a.im + b.im};
}

// Segment map (A, F, G).
template <class T>
struct Seg {
  C<T> a, f, g;
};
template <class T>
__device__ __forceinline__ Seg<T> seg_identity() {
  return {{T(1), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
}
// left then right
template <class T>
__device__ __forceinline__ Seg<T> compose(const Seg<T>& l, const Seg<T>& r) {
  return {cmul(l.a, r.a), cfma(r.a, l.f, r.f), cfma(l.a, r.g, l.g)};
}

template <class T>
__device__ __forceinline__ T shfl_up(T v, int o) { return __shfl_up(v, (unsigned)o, kWave); }
template <class T>
__device__ __forceinline__ T shfl_down(T v, int o) { return __shfl_down(v, (unsigned)o, kWave); }

// Number of Taylor terms that make the truncation error of exp on
// |w| <= kFastR fall below the type's rounding unit.
template <class T> struct Taylor;
template <> struct Taylor<double> { static constexpr int kDegree = 8; };   // (1/16)^9/9! = 4e-17
template <> struct Taylor<float> { static constexpr int kDegree = 5; };    // (1/16)^6/6! = 8e-11

template <class T>
__device__ __forceinline__ T exp_t(T v);
template <>
__device__ __forceinline__ double exp_t(double v) { return exp(v); }
template <>
__device__ __forceinline__ float exp_t(float v) { return expf(v); }
template <class T>
__device__ __forceinline__ void sincos_t(T v, T* s, T* c);
template <>
__device__ __forceinline__ void sincos_t(double v, double* s, double* c) { sincos(v, s, c); }
template <>
__device__ __forceinline__ void sincos_t(float v, float* s, float* c) { sincosf(v, s, c); }

// Per-mode constants held uniformly by the whole block.
template <class T>
struct ModeConst {
  C<T> coef[Taylor<T>::kDegree + 1];  // (-tau)^m / m!
  T tau_re, tau_im, om_re, om_im, dz_fast;
};

template <class T>
__device__ __forceinline__ ModeConst<T> mode_const(const Modes& md, int k) {
  ModeConst<T> mc;
  const double tr = md.tau_re[k], ti = md.tau_im[k];
  double cr = 1.0, ci = 0.0;
  mc.coef[0] = {T(1), T(0)};
#pragma unroll
  for (int m = 1; m <= Taylor<T>::kDegree; ++m) {
    // c_m = c_{m-1} * (-tau) / m
    const double nr = (-tr * cr + ti * ci) / m;
    const double ni = (-tr * ci - ti * cr) / m;
    cr = nr;
    ci = ni;
    mc.coef[m] = {T(cr), T(ci)};
  }
  mc.tau_re = T(tr);
  mc.tau_im = T(ti);
  mc.om_re = T(md.om_re[k]);
  mc.om_im = T(md.om_im[k]);
  mc.dz_fast = T(md.dz_fast[k]);
  return mc;
}

// e = exp(-tau dz) for dz >= 0.  Small arguments (|tau dz| <= kFastR, the
// usual case: consecutive sorted points are close on the scale sqrt(delta))
// use the Taylor polynomial in the real variable dz with complex
// coefficients; larger ones the library exp and sincos.
template <class T>
__device__ __forceinline__ C<T> exp_neg(const ModeConst<T>& mc, T dz) {
  if (dz <= mc.dz_fast) {
    constexpr int D = Taylor<T>::kDegree;
    C<T> p = mc.coef[D];
#pragma unroll
    for (int m = D - 1; m >= 0; --m) {
      p.re = fma(p.re, dz, mc.coef[m].re);
      p.im = fma(p.im, dz, mc.coef[m].im);
    }
    return p;
  }
  const T mag = exp_t(-mc.tau_re * dz);
  T s, c;
  sincos_t(mc.tau_im * dz, &s, &c);
  return {mag * c, -mag * s};
}

template <class T>
struct Staged {
  T z[kScanTile + kScanTile / kScanChunk];
  T b[kScanTile + kScanTile / kScanChunk];
  uint32_t slot[kScanTile + kScanTile / kScanChunk];   // output index; kNoSlot for a source
};

__device__ __forceinline__ int lds_pos(int e) { return e + e / kScanChunk; }
constexpr uint32_t kNoSlot = 0xffffffffu;

// Tile kernel.  FINAL = false: write the tile's (A, F, G) per mode.
// FINAL = true: read the tile's carries, run both sweeps, write u.
template <class T, int NM, bool FINAL>
__global__ __launch_bounds__(kScanThreads) void k_tiles(
    const void* keys0, const void* keys1, const uint32_t* idx0, const uint32_t* idx1,
    const PassInfo* __restrict__ pass, const T* __restrict__ alpha, int64_t N, int64_t P, Modes md,
    T* __restrict__ agg, const T* __restrict__ carry, T* __restrict__ u) {
  using K = typename KeyOf<T>::type;
  // The sorted keys sit in whichever buffer the last radix pass wrote.
  const int fb = pass->final_buf;
  const K* __restrict__ keys = (const K*)(fb ? keys1 : keys0);
  const uint32_t* __restrict__ idx = fb ? idx1 : idx0;
  __shared__ Staged<T> st;
  __shared__ Seg<T> wtot[NM][kScanWaves][2];   // per wave: [0] forward total, [1] backward total
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int64_t tile = blockIdx.x;
  const int64_t t0 = tile * kScanTile;

  // Stage the tile: coalesced reads of keys and payloads, gather alpha.
  for (int e = tid; e < kScanTile; e += kScanThreads) {
    const int64_t p = t0 + e;
    T z = T(0), b = T(0);
    uint32_t slot = kNoSlot;
    if (p < P) {
      z = from_key(keys[p]);
      const uint32_t id = idx[p];
      if ((int64_t)id < N)
        b = alpha[id];
      else if ((int64_t)id < P)
        slot = (uint32_t)((int64_t)id - N);
    }
    const int q = lds_pos(e);
    st.z[q] = z;
    st.b[q] = b;
    st.slot[q] = slot;
  }
  T zprev = T(0);
  if (tid == 0) zprev = t0 > 0 ? from_key(keys[t0 - 1]) : T(0);
  __syncthreads();

  // This thread's chunk: gaps dz_j = z_j - z_{j-1} and strengths b_j.
  const int e0 = tid * kScanChunk;
  T dz[kScanChunk], bb[kScanChunk];
  {
    const int64_t valid = P - t0;   // points of this tile that exist
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
    }
  }

  T acc[kScanChunk];
#pragma unroll
  for (int j = 0; j < kScanChunk; ++j) acc[j] = T(0);

#pragma unroll 1
  for (int k = 0; k < NM; ++k) {
    const ModeConst<T> mc = mode_const<T>(md, k);
    C<T> ex[kScanChunk];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) ex[j] = exp_neg(mc, dz[j]);

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

    // Tile totals (reduce) or carries into this chunk (final).
    if (!FINAL) {
      if (tid == 0) {
        Seg<T> tot = seg_identity<T>();
        Seg<T> totb = seg_identity<T>();
        for (int w = 0; w < kScanWaves; ++w) {
          const Seg<T> fw = wtot[k][w][0];
          const Seg<T> bw = wtot[k][w][1];
          tot.f = cfma(fw.a, tot.f, fw.f);
          tot.a = cmul(tot.a, fw.a);
          totb.g = cfma(totb.a, bw.g, totb.g);
          totb.a = cmul(totb.a, bw.a);
        }
        T* o = agg + ((size_t)tile * NM + k) * 6;
        o[0] = tot.a.re; o[1] = tot.a.im;
        o[2] = tot.f.re; o[3] = tot.f.im;
        o[4] = totb.g.re; o[5] = totb.g.im;
      }
    } else {
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
        acc[j] = fma(mc.om_re, h.re, fma(-mc.om_im, h.im, acc[j]));
      }
      // Backward sweep: h- (exclusive) at every point.
      C<T> g = cb;
#pragma unroll
      for (int j = kScanChunk - 1; j >= 0; --j) {
        acc[j] = fma(mc.om_re, g.re, fma(-mc.om_im, g.im, acc[j]));
        g = cmul(ex[j], cadd(g, C<T>{bb[j], T(0)}));
      }
    }
  }

  if (FINAL) {
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      const uint32_t slot = st.slot[lds_pos(e0 + j)];
      if ((int64_t)slot < P - N) u[slot] = acc[j];
    }
  }
}

// Carries over tiles for mode blockIdx.x: CF[t] = forward value entering tile
// t from the left (h+ at the point before it), CB[t] = backward value
// entering from the right (h- at its last point).
template <class T, int NM>
__global__ __launch_bounds__(kCarryThreads) void k_carry(const T* __restrict__ agg, int64_t tiles,
                                                         T* __restrict__ carry) {
  constexpr int W = kCarryThreads / kWave;
  __shared__ Seg<T> wf[W], wb[W];
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int wave = tid / kWave;
  const int64_t per = (tiles + kCarryThreads - 1) / kCarryThreads;
  const int64_t a0 = (int64_t)tid * per;
  const int64_t a1 = a0 + per < tiles ? a0 + per : tiles;

  auto tile_seg = [&](int64_t t) {
    const T* p = agg + ((size_t)t * NM + k) * 6;
    Seg<T> s;
    s.a = {p[0], p[1]};
    s.f = {p[2], p[3]};
    s.g = {p[4], p[5]};
    return s;
  };
  // Fold this thread's tiles.
  Seg<T> mine = seg_identity<T>();
  for (int64_t t = a0; t < a1; ++t) mine = compose(mine, tile_seg(t));

  Seg<T> pf = mine, sb = mine;
  for (int o = 1; o < kWave; o <<= 1) {
    Seg<T> l, r;
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
  if (lane == kWave - 1) wf[wave] = pf;
  if (lane == 0) wb[wave] = sb;
  __syncthreads();

  C<T> cf = {T(0), T(0)};
  C<T> cb = {T(0), T(0)};
  for (int w = 0; w < wave; ++w) cf = cfma(wf[w].a, cf, wf[w].f);
  for (int w = W - 1; w > wave; --w) cb = cfma(wb[w].a, cb, wb[w].g);
  Seg<T> xl, xr;
  xl.a.re = shfl_up(pf.a.re, 1); xl.a.im = shfl_up(pf.a.im, 1);
  xl.f.re = shfl_up(pf.f.re, 1); xl.f.im = shfl_up(pf.f.im, 1);
  xr.a.re = shfl_down(sb.a.re, 1); xr.a.im = shfl_down(sb.a.im, 1);
  xr.g.re = shfl_down(sb.g.re, 1); xr.g.im = shfl_down(sb.g.im, 1);
  if (lane > 0) cf = cfma(xl.a, cf, xl.f);
  if (lane < kWave - 1) cb = cfma(xr.a, cb, xr.g);

  for (int64_t t = a0; t < a1; ++t) {
    T* o = carry + ((size_t)t * NM + k) * 4;
    o[0] = cf.re;
    o[1] = cf.im;
    const Seg<T> s = tile_seg(t);
    cf = cfma(s.a, cf, s.f);
  }
  for (int64_t t = a1 - 1; t >= a0; --t) {
    T* o = carry + ((size_t)t * NM + k) * 4;
    o[2] = cb.re;
    o[3] = cb.im;
    const Seg<T> s = tile_seg(t);
    cb = cfma(s.a, cb, s.g);
  }
}

template <class T>
__global__ void k_fill_zero(T* __restrict__ u, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) u[i] = T(0);
}

template <class T, int NM>
hipError_t scan_nm(const Workspace& w, const Modes& md, const T* alpha, int64_t M, int64_t N, T* u,
                   hipStream_t s, Timeline* tl) {
  const int64_t P = M + N;
  const dim3 grid((unsigned)w.scan_tiles);
  hipLaunchKernelGGL((k_tiles<T, NM, false>), grid, dim3(kScanThreads), 0, s, w.keys[0], w.keys[1],
                     w.idx[0], w.idx[1], w.pass, alpha, N, P, md, (T*)w.agg, (const T*)w.carry, u);
  tl->mark(s);
  hipLaunchKernelGGL((k_carry<T, NM>), dim3(NM), dim3(kCarryThreads), 0, s, (const T*)w.agg,
                     w.scan_tiles, (T*)w.carry);
  tl->mark(s);
  hipLaunchKernelGGL((k_tiles<T, NM, true>), grid, dim3(kScanThreads), 0, s, w.keys[0], w.keys[1],
                     w.idx[0], w.idx[1], w.pass, alpha, N, P, md, (T*)w.agg, (const T*)w.carry, u);
  tl->mark(s);
  return hipGetLastError();
}

}  // namespace

template <class T>
hipError_t scan_points(const Workspace& w, const Modes& md, const T* alpha, int64_t M, int64_t N,
                       T* u, hipStream_t s, Timeline* tl) {
  switch (md.n) {
    case 1: return scan_nm<T, 1>(w, md, alpha, M, N, u, s, tl);
    case 2: return scan_nm<T, 2>(w, md, alpha, M, N, u, s, tl);
    case 3: return scan_nm<T, 3>(w, md, alpha, M, N, u, s, tl);
    case 4: return scan_nm<T, 4>(w, md, alpha, M, N, u, s, tl);
    case 5: return scan_nm<T, 5>(w, md, alpha, M, N, u, s, tl);
    case 6: return scan_nm<T, 6>(w, md, alpha, M, N, u, s, tl);
    case 7: return scan_nm<T, 7>(w, md, alpha, M, N, u, s, tl);
    case 8: return scan_nm<T, 8>(w, md, alpha, M, N, u, s, tl);
    default: return hipErrorInvalidValue;
  }
}

template <class T>
hipError_t fill_zero(T* u, int64_t n, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill_zero<T>, dim3((unsigned)blocks), dim3(256), 0, s, u, n);
  return hipGetLastError();
}

template hipError_t scan_points<double>(const Workspace&, const Modes&, const double*, int64_t,
                                        int64_t, double*, hipStream_t, Timeline*);
template hipError_t scan_points<float>(const Workspace&, const Modes&, const float*, int64_t,
                                       int64_t, float*, hipStream_t, Timeline*);
template hipError_t fill_zero<double>(double*, int64_t, hipStream_t);
template hipError_t fill_zero<float>(float*, int64_t, hipStream_t);

}  // namespace fgt
