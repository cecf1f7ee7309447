// Small transforms (P = M + N <= kSmallMax): the whole of fgt_eval -- the
// merged ascending sort of Section 4, the forward and backward recurrences
// (4.5)-(4.6) of every mode and the sum Re(omega_k (h+ + h-)) at the targets
// (4.1), (4.4) -- in two launches, with the points held in LDS: one workgroup
// per mode, each sorting the points itself and writing its mode's sums, then
// a sum over the modes in mode order (the same bits on every run) scattered to
// the targets.  At these sizes the multi-kernel path is bound by the latency
// of its ~20 launches rather than by any one of them.
//
//   keys   IEEE order keys of [y; x] (-0 read as +0) beside their merged indices;
//   sort   a bitonic network over (key, index) pairs padded to a power of two:
//          comparing the index on equal keys gives the stable order, so a
//          source coinciding with a target comes first, the split (4.4) assumes;
//   scan   each thread owns kSmallPer consecutive sorted points; per mode the
//          threads' chunk maps (A, F, G) are scanned over the wave and the
//          waves' totals are composed in order, then each thread sweeps its
//          chunk in both directions.
// The sorted coordinates, merged ids and strengths are left in the workspace
// (by the first workgroup) as the multi-kernel path leaves them, so
// fgt_eval_sorted and fgt_backward with FGT_SORTED start from them.  The sort
// here is exact (every key bit).
#include "fgt_device.h"

namespace fgt {
namespace {

constexpr int kSmallThreads = 1024;
constexpr int kSmallPer = kSmallMax / kSmallThreads;
constexpr int kSmallWaves = kSmallThreads / kWave;

// exp(-tau dz) for a thread's gaps: the Taylor polynomial of the wave's degree
// (the smallest whose truncation at the wave's largest gap is below the unit
// roundoff), the library functions for gaps beyond its range.
template <class T>
__device__ __forceinline__ void small_exps(const Modes& md, int k, const T* dz, T dzmax,
                                           C<T>* ex) {
  const double rr = md.tau_abs[k] * (double)dzmax;
  int D = kTaylorMax;
#pragma unroll
  for (int d = kTaylorMax; d >= 1; --d)
    if (rr <= md.taylor_thr[d]) D = d;
#pragma unroll
  for (int j = 0; j < kSmallPer; ++j) ex[j] = {T(0), T(0)};
#pragma unroll
  for (int m = kTaylorMax; m >= 0; --m) {
    if (m <= D) {
      const T c_re = T(md.coef_re[k][m]), c_im = T(md.coef_im[k][m]);
#pragma unroll
      for (int j = 0; j < kSmallPer; ++j) {
        ex[j].re = fma(ex[j].re, dz[j], c_re);
        ex[j].im = fma(ex[j].im, dz[j], c_im);
      }
    }
  }
  const T dz_lim = T(md.dz_lim[k]);
#pragma unroll
  for (int j = 0; j < kSmallPer; ++j)
    if (dz[j] > dz_lim) ex[j] = exp_neg_general<T>(T(md.tau_re[k]), T(md.tau_im[k]), dz[j]);
}

// Block k: the sort, then mode k's sums at every sorted point into part[k][P].
template <class T>
__global__ __launch_bounds__(kSmallThreads) void k_small(
    const T* __restrict__ x, int64_t M, const T* __restrict__ y, const T* __restrict__ alpha,
    int64_t N, Modes md, T* __restrict__ part, T* __restrict__ zs, uint32_t* __restrict__ ids,
    T* __restrict__ bs, PassInfo* __restrict__ pass, uint32_t* __restrict__ status) {
  using K = typename KeyOf<T>::type;
  __shared__ K skey[kSmallMax];
  __shared__ uint32_t sid[kSmallMax];
  __shared__ Seg<T> wtot[kSmallWaves][2];   // per wave: forward and backward totals
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int wave = tid / kWave;
  const int P = (int)(M + N);
  int Pp = 2;
  while (Pp < P) Pp <<= 1;

  if (tid == 0) s_bad = 0;
  __syncthreads();
  bool bad = false;
  for (int p = tid; p < Pp; p += kSmallThreads) {
    if (p < P) {
      const T z = p < N ? y[p] : x[p - N];
      bad |= !isfinite(z);
      skey[p] = to_key(z);
      sid[p] = (uint32_t)p;
    } else {
      skey[p] = ~K(0);   // padding sorts last
      sid[p] = kNoSlot;
    }
  }
  if (bad) atomicOr(&s_bad, 1);
  __syncthreads();

  // Bitonic network, ascending in (key, merged index).  Pair t of a stage
  // joins elements i and i + j; the 64 pairs of a wave lie in one block of 128
  // elements while j <= 64, so between two such stages the wave's own LDS order
  // suffices and only stages with partners further apart need the block barrier.
  for (int k = 2; k <= Pp; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = tid; t < Pp / 2; t += kSmallThreads) {
        const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int l = i + j;
        const K ki = skey[i], kl = skey[l];
        const uint32_t ii = sid[i], il = sid[l];
        const bool l_first = kl < ki || (kl == ki && il < ii);
        if (l_first == ((i & k) == 0)) {
          skey[i] = kl;
          skey[l] = ki;
          sid[i] = il;
          sid[l] = ii;
        }
      }
      const int j_next = j > 1 ? j >> 1 : k;   // the next stage's distance (k << 1 >> 1)
      if (j >= 2 * kWave || j_next >= 2 * kWave)
        __syncthreads();
      else
        __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();

  // The thread's points: coordinates, gaps, strengths; the first block writes
  // the sorted state to the workspace.
  const bool first = blockIdx.x == 0;
  const int p0 = tid * kSmallPer;
  T dz[kSmallPer], bb[kSmallPer], acc[kSmallPer];
  uint32_t id[kSmallPer];
  T zl = p0 > 0 && p0 - 1 < P ? from_key(skey[p0 - 1]) : T(0);
  T dzmax = T(0);
#pragma unroll
  for (int c = 0; c < kSmallPer; ++c) {
    const int p = p0 + c;
    const bool valid = p < P;
    const T z = valid ? from_key(skey[p]) : T(0);
    id[c] = valid ? sid[p] : kNoSlot;
    bb[c] = (valid && id[c] < (uint32_t)N) ? alpha[id[c]] : T(0);
    dz[c] = (valid && p > 0) ? z - zl : T(0);
    zl = valid ? z : zl;
    dzmax = dz[c] > dzmax ? dz[c] : dzmax;
    acc[c] = T(0);
    if (valid && first) {
      zs[p] = z;
      ids[p] = id[c];
      bs[p] = bb[c];
    }
  }
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const T other = shfl_xor(dzmax, o);
    dzmax = other > dzmax ? other : dzmax;
  }

  {
    const int k = blockIdx.x;
    C<T> ex[kSmallPer];
    small_exps(md, k, dz, dzmax, ex);
    // Chunk map: A = prod e, F = forward fold from 0, G = backward fold from 0.
    Seg<T> s;
    s.a = ex[0];
    s.f = {bb[0], T(0)};
#pragma unroll
    for (int c = 1; c < kSmallPer; ++c) {
      s.a = cmul(s.a, ex[c]);
      s.f = cfma(ex[c], s.f, C<T>{bb[c], T(0)});
    }
    s.g = {T(0), T(0)};
#pragma unroll
    for (int c = kSmallPer - 1; c >= 0; --c) s.g = cmul(ex[c], cadd(s.g, C<T>{bb[c], T(0)}));
    Seg<T> pf, sb;
    wave_scans(s, lane, pf, sb);
    if (lane == kWave - 1) wtot[wave][0] = pf;
    if (lane == 0) wtot[wave][1] = sb;
    __syncthreads();
    // h+ before the chunk and h- at its last point: earlier (later) waves in
    // order, then the earlier (later) lanes of this wave.
    C<T> cf = {T(0), T(0)}, cb = {T(0), T(0)};
    for (int w = 0; w < wave; ++w) cf = cfma(wtot[w][0].a, cf, wtot[w][0].f);
    for (int w = kSmallWaves - 1; w > wave; --w) cb = cfma(wtot[w][1].a, cb, wtot[w][1].g);
    Seg<T> xl, xr;
    xl.a.re = shfl_up(pf.a.re, 1); xl.a.im = shfl_up(pf.a.im, 1);
    xl.f.re = shfl_up(pf.f.re, 1); xl.f.im = shfl_up(pf.f.im, 1);
    xr.a.re = shfl_down(sb.a.re, 1); xr.a.im = shfl_down(sb.a.im, 1);
    xr.g.re = shfl_down(sb.g.re, 1); xr.g.im = shfl_down(sb.g.im, 1);
    if (lane > 0) cf = cfma(xl.a, cf, xl.f);
    if (lane < kWave - 1) cb = cfma(xr.a, cb, xr.g);
    const T om_re = T(md.om_re[k]), om_im = T(md.om_im[k]);
    C<T> h = cf;
#pragma unroll
    for (int c = 0; c < kSmallPer; ++c) {
      h = cfma(ex[c], h, C<T>{bb[c], T(0)});
      acc[c] = fma(om_re, h.re, fma(-om_im, h.im, acc[c]));
    }
    C<T> g = cb;
#pragma unroll
    for (int c = kSmallPer - 1; c >= 0; --c) {
      acc[c] = fma(om_re, g.re, fma(-om_im, g.im, acc[c]));
      g = cmul(ex[c], cadd(g, C<T>{bb[c], T(0)}));
    }
  }

  T* __restrict__ mine = part + (size_t)blockIdx.x * (size_t)P;
#pragma unroll
  for (int c = 0; c < kSmallPer; ++c)
    if (p0 + c < P) mine[p0 + c] = acc[c];
  if (first && tid == 0) {
    *status = s_bad ? kStatusNonFinite : 0u;
    pass->final_buf = 0;
    pass->last_pass = -1;
  }
}

// u at the targets: the modes' sums added in mode order.
template <class T>
__global__ __launch_bounds__(256) void k_small_sum(const uint32_t* __restrict__ ids,
                                                   const T* __restrict__ part, int nm, int64_t P,
                                                   int64_t N, T* __restrict__ u) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const uint32_t id = ids[p];
  if (id < (uint32_t)N) return;   // a source
  T acc = part[p];
  for (int k = 1; k < nm; ++k) acc += part[(size_t)k * (size_t)P + p];
  u[id - (uint32_t)N] = acc;
}

}  // namespace

// fgt_eval for P = M + N <= kSmallMax in two launches, one phase on tl; *done
// is false (and nothing is enqueued or recorded) for larger problems.
template <class T>
hipError_t small_eval(const Workspace& w, const Modes& md, const T* x, int64_t M, const T* y,
                      const T* alpha, int64_t N, T* u, hipStream_t s, Timeline* tl, bool* done) {
  *done = false;
  if (M + N > kSmallMax || M <= 0 || N <= 0) return hipSuccess;
  if (md.n < 1 || md.n > FGT_MAX_MODES || !w.small_part) return hipErrorInvalidValue;
  *done = true;
  const int64_t P = M + N;
  tl->mark(s);
  hipLaunchKernelGGL(k_small<T>, dim3((unsigned)md.n), dim3(kSmallThreads), 0, s, x, M, y, alpha,
                     N, md, (T*)w.small_part, (T*)w.keys[0], w.ids, (T*)w.b, w.pass, w.status);
  hipLaunchKernelGGL(k_small_sum<T>, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s,
                     (const uint32_t*)w.ids, (const T*)w.small_part, md.n, P, N, (T*)u);
  tl->mark(s);
  return hipGetLastError();
}

template hipError_t small_eval<double>(const Workspace&, const Modes&, const double*, int64_t,
                                       const double*, const double*, int64_t, double*,
                                       hipStream_t, Timeline*, bool*);
template hipError_t small_eval<float>(const Workspace&, const Modes&, const float*, int64_t,
                                      const float*, const float*, int64_t, float*, hipStream_t,
                                      Timeline*, bool*);

}  // namespace fgt
