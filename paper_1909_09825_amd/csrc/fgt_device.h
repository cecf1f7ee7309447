// Device helpers shared by the single-transform and batched scans: complex
// arithmetic, segment maps of the affine recurrences and their composition,
// wave shuffles, the general complex exponential, and the tile-carry kernels.
#pragma once

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
template <class T>
__device__ __forceinline__ T shfl_xor(T v, int o) { return __shfl_xor(v, o, kWave); }

// Inclusive sum over the wave's lanes in registers (DPP): Hillis-Steele steps
// of 1, 2, 4 and 8 lanes inside each row of 16 (row_shr), then the totals of
// rows 0 and 2 into rows 1 and 3 (row_bcast:15) and of rows 0-1 into rows
// 2-3 (row_bcast:31).  A lane whose source is outside its row, or whose row
// is masked out, receives 0 (the `old` operand, bound_ctrl off), so it adds
// nothing.  64-bit values move as two 32-bit halves.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
// Row shift: lanes shifted in from outside the row read 0 (bound_ctrl), so
// no zero source register is needed.
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <class T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
  v += dpp_shift<0x111>(v);       // row_shr:1
  v += dpp_shift<0x112>(v);       // row_shr:2
  v += dpp_shift<0x114>(v);       // row_shr:4
  v += dpp_shift<0x118>(v);       // row_shr:8
  v += dpp_move<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}
// Lane l's value, in every lane (a scalar read).
__device__ __forceinline__ double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
// The sum over the whole wave, in every lane.
template <class T>
__device__ __forceinline__ T wave_total(T v) {
  return lane_value(wave_inclusive_sum(v), kWave - 1);
}

template <class T> struct Prec;
template <> struct Prec<double> { static constexpr double kUnit = 1.1102230246251565e-16; };  // 2^-53
template <> struct Prec<float> { static constexpr double kUnit = 5.9604644775390625e-08; };    // 2^-24

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

// exp(-tau x) through the library exp and sincos; kept out of line so the
// rare large-argument case does not cost registers in the hot loops.
template <class T>
__device__ __noinline__ C<T> exp_neg_general(T tr, T ti, T x) {
  const T mag = exp_t(-tr * x);
  T s, c;
  sincos_t(ti * x, &s, &c);
  return {mag * c, -mag * s};
}

// 1/m! for the moment sums.
struct InvFact {
  double v[kMomentMax + 1];
  constexpr InvFact() : v() {
    double f = 1.0;
    for (int m = 0; m <= kMomentMax; ++m) {
      if (m > 0) f *= m;
      v[m] = 1.0 / f;
    }
  }
};
__constant__ constexpr InvFact kInvFact{};

// ---------------------------------------------------------------------------
// Carries over tiles, for every scan q (one per mode; q = channel * modes +
// mode when two strength channels share the sweeps).  CF[t] = forward value
// entering tile t from the left (h+ at the point before it), CB[t] = backward
// value entering from the right (h- at its last point).  Three levels so that
// the whole chip takes part: tiles are grouped in chunks of 64 (one block per
// chunk, one wave per scan at a time),
//   k_carry_up    the composed map of each chunk,
//   k_carry_top   per scan, the values entering each chunk (sequential runs
//                 per thread, then a block scan),
//   k_carry_down  per chunk, the values entering each of its tiles.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ Seg<T> load_seg(const T* __restrict__ p) {
  Seg<T> s;
  s.a = {p[0], p[1]};
  s.f = {p[2], p[3]};
  s.g = {p[4], p[5]};
  return s;
}

// Inclusive prefix (pf: A, F) and suffix (sb: A, G) of the lanes' maps.
template <class T>
__device__ __forceinline__ void wave_scans(const Seg<T>& s, int lane, Seg<T>& pf, Seg<T>& sb) {
  pf = s;
  sb = s;
#pragma unroll
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
}

// Tile maps of the single-transform scan: [tile][q][kAggStride].
template <class T>
struct AggMaps {
  const T* agg;
  int nq;
  __device__ __forceinline__ Seg<T> operator()(int64_t t, int q) const {
    return load_seg(agg + ((size_t)t * nq + q) * kAggStride);
  }
};

// Tile maps of the batched scan: A per (tile, mode) in a[(t * nm + k) * 2],
// F and G per (tile, mode, column) in fg[(t * nq + q) * 4], q = k * R + column.
template <class T>
struct BatchMaps {
  const T* a;
  const T* fg;
  int nm, R;
  __device__ __forceinline__ Seg<T> operator()(int64_t t, int q) const {
    const T* pa = a + ((size_t)t * nm + q / R) * 2;
    const T* pf = fg + ((size_t)t * nm * R + q) * 4;
    Seg<T> s;
    s.a = {pa[0], pa[1]};
    s.f = {pf[0], pf[1]};
    s.g = {pf[2], pf[3]};
    return s;
  }
};

// k_carry_up and k_carry_down take one chunk of 64 tiles per block and loop
// over the scans, one wave per scan at a time: the maps of a tile lie together
// (all scans of a tile in one row), so the rows a block reads stay in cache
// while its waves walk through the scans.
constexpr int kCarryWaves = 4;

template <class T, class Maps>
__global__ __launch_bounds__(kWave * kCarryWaves) void k_carry_up(Maps maps, int64_t tiles, int nq,
                                                                  T* __restrict__ chunk_agg) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int64_t chunk = blockIdx.x;
  const int64_t t = chunk * kWave + lane;
  for (int q = wave; q < nq; q += kCarryWaves) {
    const Seg<T> s = t < tiles ? maps(t, q) : seg_identity<T>();
    Seg<T> pf, sb;
    wave_scans(s, lane, pf, sb);
    T* o = chunk_agg + ((size_t)chunk * nq + q) * 6;
    if (lane == kWave - 1) {
      o[0] = pf.a.re; o[1] = pf.a.im;
      o[2] = pf.f.re; o[3] = pf.f.im;
    }
    if (lane == 0) {
      o[4] = sb.g.re; o[5] = sb.g.im;
    }
  }
}

template <class T>
__global__ __launch_bounds__(kCarryThreads) void k_carry_top(const T* __restrict__ chunk_agg,
                                                             int64_t chunks, int nq,
                                                             T* __restrict__ chunk_carry) {
  constexpr int W = kCarryThreads / kWave;
  __shared__ Seg<T> wf[W], wb[W];
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int wave = tid / kWave;
  const int64_t per = (chunks + kCarryThreads - 1) / kCarryThreads;
  const int64_t a0 = (int64_t)tid * per;
  const int64_t a1 = a0 + per < chunks ? a0 + per : chunks;
  auto seg = [&](int64_t c) { return load_seg(chunk_agg + ((size_t)c * nq + q) * 6); };

  Seg<T> mine = seg_identity<T>();
  for (int64_t c = a0; c < a1; ++c) mine = compose(mine, seg(c));
  Seg<T> pf, sb;
  wave_scans(mine, lane, pf, sb);
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

  for (int64_t c = a0; c < a1; ++c) {
    T* o = chunk_carry + ((size_t)c * nq + q) * 4;
    o[0] = cf.re;
    o[1] = cf.im;
    const Seg<T> s = seg(c);
    cf = cfma(s.a, cf, s.f);
  }
  for (int64_t c = a1 - 1; c >= a0; --c) {
    T* o = chunk_carry + ((size_t)c * nq + q) * 4;
    o[2] = cb.re;
    o[3] = cb.im;
    const Seg<T> s = seg(c);
    cb = cfma(s.a, cb, s.g);
  }
}

template <class T, class Maps>
__global__ __launch_bounds__(kWave * kCarryWaves) void k_carry_down(
    Maps maps, int64_t tiles, int nq, const T* __restrict__ chunk_carry, T* __restrict__ carry) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int64_t chunk = blockIdx.x;
  const int64_t t = chunk * kWave + lane;
  for (int q = wave; q < nq; q += kCarryWaves) {
    const Seg<T> s = t < tiles ? maps(t, q) : seg_identity<T>();
    Seg<T> pf, sb;
    wave_scans(s, lane, pf, sb);
    const T* cc = chunk_carry + ((size_t)chunk * nq + q) * 4;
    C<T> cf = {cc[0], cc[1]};
    C<T> cb = {cc[2], cc[3]};
    // exclusive: the tiles before / after this one inside the chunk
    Seg<T> xl, xr;
    xl.a.re = shfl_up(pf.a.re, 1); xl.a.im = shfl_up(pf.a.im, 1);
    xl.f.re = shfl_up(pf.f.re, 1); xl.f.im = shfl_up(pf.f.im, 1);
    xr.a.re = shfl_down(sb.a.re, 1); xr.a.im = shfl_down(sb.a.im, 1);
    xr.g.re = shfl_down(sb.g.re, 1); xr.g.im = shfl_down(sb.g.im, 1);
    if (lane > 0) cf = cfma(xl.a, cf, xl.f);
    if (lane < kWave - 1) cb = cfma(xr.a, cb, xr.g);
    if (t < tiles) {
      T* o = carry + ((size_t)t * nq + q) * 4;
      o[0] = cf.re;
      o[1] = cf.im;
      o[2] = cb.re;
      o[3] = cb.im;
    }
  }
}

// Launch the three carry levels for nq scans over `tiles` tiles.
template <class T, class Maps>
hipError_t launch_carries(const Maps& maps, int64_t tiles, int nq, T* chunk_agg, T* chunk_carry,
                          T* carry, hipStream_t s) {
  const int64_t chunks = (tiles + kWave - 1) / kWave;
  hipLaunchKernelGGL((k_carry_up<T, Maps>), dim3((unsigned)chunks), dim3(kWave * kCarryWaves), 0, s,
                     maps, tiles, nq, chunk_agg);
  hipLaunchKernelGGL(k_carry_top<T>, dim3((unsigned)nq), dim3(kCarryThreads), 0, s,
                     (const T*)chunk_agg, chunks, nq, chunk_carry);
  hipLaunchKernelGGL((k_carry_down<T, Maps>), dim3((unsigned)chunks), dim3(kWave * kCarryWaves), 0,
                     s, maps, tiles, nq, (const T*)chunk_carry, carry);
  return hipGetLastError();
}

}  // namespace
}  // namespace fgt
