// C ABI of the fast Gauss transform: plans, validation, workspace layout and
// the launch sequence sort -> scan on the caller's stream.
#include <math.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fgt_internal.h"

namespace fgt {

typedef SoeTable fgt_soe_table_t;
#include "soe_tables.inc"

namespace {

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Largest digits served per element type: FP64 up to the most accurate
// shipped table, FP32 up to 6 digits (its rounding unit is 6e-8).
int max_digits_f64() {
  int best = 0;
  for (int i = 0; i < FGT_SOE_NUM_TABLES; ++i) {
    int d = (int)floor(-log10(kSoeTables[i].err_bound));
    if (d > best) best = d;
  }
  return best;
}

}  // namespace

Workspace layout(void* base, int64_t P, int esz, int n_modes) {
  Workspace w;
  memset(&w, 0, sizeof(w));
  const int digits = esz == 8 ? 8 : 4;
  w.sort_tiles = (P + kSortTile - 1) / kSortTile;
  w.scan_tiles = (P + kScanTile - 1) / kScanTile;
  w.wave_tiles = (P + kWTile - 1) / kWTile;
  if (w.sort_tiles < 1) w.sort_tiles = 1;
  if (w.scan_tiles < 1) w.scan_tiles = 1;
  if (w.wave_tiles < 1) w.wave_tiles = 1;
  char* b = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? (void*)(b + off) : nullptr;
    off += align_up(bytes);
    return p;
  };
  // The region cleared at the start of each call is contiguous: status word
  // (always at offset 0), histograms, tile counters and the first look-back buffer.
  w.status = (uint32_t*)take(sizeof(uint32_t) * 64);
  w.range = (unsigned long long*)take(3 * sizeof(unsigned long long));
  w.hist = (uint32_t*)take(sizeof(uint32_t) * digits * kSortRadix);
  w.tile_ctr = (uint32_t*)take(sizeof(uint32_t) * 8);
  w.lookback[0] = (uint64_t*)take(sizeof(uint64_t) * (size_t)w.sort_tiles * kSortRadix);
  w.zero_bytes = off;
  w.lookback[1] = (uint64_t*)take(sizeof(uint64_t) * (size_t)w.sort_tiles * kSortRadix);
  w.dig_off = (uint32_t*)take(sizeof(uint32_t) * digits * kSortRadix);
  w.pass = (PassInfo*)take(sizeof(PassInfo));
  // Scan state: the forward's n_modes scans over wave_tiles tiles, or the
  // adjoint's 2 x n_modes scans (two strength channels) over scan_tiles tiles.
  const size_t nm = (size_t)n_modes;
  const size_t tq_fwd = nm * (size_t)w.wave_tiles;
  const size_t tq_adj = 2 * nm * (size_t)w.scan_tiles;
  const size_t tq = tq_fwd > tq_adj ? tq_fwd : tq_adj;
  const size_t cq_fwd = nm * (size_t)((w.wave_tiles + kWave - 1) / kWave);
  const size_t cq_adj = 2 * nm * (size_t)((w.scan_tiles + kWave - 1) / kWave);
  const size_t cq = cq_fwd > cq_adj ? cq_fwd : cq_adj;
  w.agg = take((size_t)esz * kAggStride * tq);
  w.tile_k = (int32_t*)take(sizeof(int32_t) * (size_t)(w.wave_tiles > w.scan_tiles ? w.wave_tiles
                                                                                  : w.scan_tiles));
  w.carry = take((size_t)esz * 4 * tq);
  w.chunk_agg = take((size_t)esz * 6 * cq);
  w.chunk_carry = take((size_t)esz * 4 * cq);
  w.tile_part = (double*)take(sizeof(double) * (size_t)w.scan_tiles);
  w.keys[0] = take((size_t)esz * (size_t)P);
  w.keys[1] = take((size_t)esz * (size_t)P);
  // The two permutation buffers are consecutive; after the sort they hold the
  // transposed strengths (esz * P <= 2 * align_up(4 * P) bytes).
  w.idx[0] = (uint32_t*)take(sizeof(uint32_t) * (size_t)P);
  w.idx[1] = (uint32_t*)take(sizeof(uint32_t) * (size_t)P);
  w.bt = (void*)w.idx[0];
  w.b = take((size_t)esz * (size_t)P);
  w.ids = (uint32_t*)take(sizeof(uint32_t) * (size_t)P);
  w.small_part = P <= kSmallMax ? take((size_t)esz * nm * (size_t)P) : nullptr;
  w.total = off;
  return w;
}

const SoeTable* choose_table(int digits) {
  const double target = pow(10.0, -digits);
  const SoeTable* tab = nullptr;
  for (int i = 0; i < FGT_SOE_NUM_TABLES; ++i) {
    if (kSoeTables[i].err_bound <= target && (!tab || kSoeTables[i].n_modes < tab->n_modes))
      tab = &kSoeTables[i];
  }
  return tab;
}

int max_digits(int dtype) {
  if (dtype == FGT_F64) return max_digits_f64();
  if (dtype == FGT_F32) return 6;
  return 0;
}

void make_modes(const SoeTable* tab, double delta, int dtype, Modes* m) {
  memset(m, 0, sizeof(*m));
  m->n = tab->n_modes;
  const double rs = 1.0 / sqrt(delta);
  m->tau_abs_max = 0.0;
  for (int k = 0; k < tab->n_modes; ++k) {
    m->tau_re[k] = tab->tau0_re[k] * rs;
    m->tau_im[k] = tab->tau0_im[k] * rs;
    m->om_re[k] = tab->om_re[k];
    m->om_im[k] = tab->om_im[k];
    m->tau_abs[k] = hypot(m->tau_re[k], m->tau_im[k]);
    m->dom_re[k] = -(m->tau_re[k] * tab->om_re[k] - m->tau_im[k] * tab->om_im[k]);
    m->dom_im[k] = -(m->tau_re[k] * tab->om_im[k] + m->tau_im[k] * tab->om_re[k]);
    if (m->tau_abs[k] > m->tau_abs_max) m->tau_abs_max = m->tau_abs[k];
  }
  // Sort resolution.  Two points closer than w = s_w sqrt(delta) may be left in
  // either order.  If a source at y and a target at x swap places, x - y
  // changes sign and the recurrences evaluate S at -|x - y| instead of
  // +|x - y| (continued through the same exponentials); with s = |x - y| /
  // sqrt(delta) the change is |Re sum omega (e^{tau0 s} - e^{-tau0 s})| <=
  // 2 |Re sum omega tau0| s + (1/3) sum |omega| |tau0|^3 s^3 cosh(max|tau0| s).
  // With IEEE order keys s_w makes this at most 1e-6 E_n, so the result stays
  // within (1 + 1e-6) E_n sum|alpha| of the Gauss transform.  The FP64 grid
  // code splits that allowance: unordered pairs take 0.5e-6 E_n, and moving
  // each point by at most code_tol the other half, since a shift e of both
  // ends changes a term by at most |alpha| (max|G'| + E'_n) 2 e / sqrt(delta)
  // with max|G'| = 2^{-1/2} e^{-1/2} for G(s) = exp(-s^2/4).
  {
    double slope = 0.0, c3 = 0.0, tmax = 0.0;
    for (int k = 0; k < tab->n_modes; ++k) {
      slope += tab->om_re[k] * tab->tau0_re[k] - tab->om_im[k] * tab->tau0_im[k];
      const double ta = hypot(tab->tau0_re[k], tab->tau0_im[k]);
      c3 += hypot(tab->om_re[k], tab->om_im[k]) * ta * ta * ta;
      if (ta > tmax) tmax = ta;
    }
    slope = fabs(slope);
    auto width = [&](double fraction) {
      const double target = fraction * tab->err_bound;
      double lo = 0.0, hi = 1.0;
      for (int it = 0; it < 200; ++it) {
        const double s = 0.5 * (lo + hi);
        const double b = 2.0 * slope * s + c3 * s * s * s * cosh(tmax * s) / 3.0;
        if (b <= target) lo = s; else hi = s;
      }
      return lo * sqrt(delta);
    };
    m->key_width = width(1e-6);
    m->sort.key_width = m->key_width;
    m->sort.key_width_q = width(0.5e-6);
    const double max_dg = sqrt(0.5) * exp(-0.5);
    m->sort.code_tol = 0.25e-6 * tab->err_bound * sqrt(delta) / (max_dg + tab->deriv_err_bound);
  }
  for (int k = 0; k < tab->n_modes; ++k) {
    double cr = 1.0, ci = 0.0;
    for (int j = 0; j <= kTaylorMax; ++j) {
      m->coef_re[k][j] = cr;
      m->coef_im[k][j] = ci;
      const double nr = (-m->tau_re[k] * cr + m->tau_im[k] * ci) / (j + 1);
      const double ni = (-m->tau_re[k] * ci - m->tau_im[k] * cr) / (j + 1);
      cr = nr;
      ci = ni;
    }
  }
  // Taylor thresholds for the element type's unit roundoff.
  const double unit = dtype == FGT_F64 ? ldexp(1.0, -53) : ldexp(1.0, -24);
  double fact = 1.0;
  m->taylor_thr[0] = 0.0;
  for (int d = 1; d <= kTaylorMax; ++d) {
    fact *= (d + 1);   // (d+1)!
    m->taylor_thr[d] = pow(unit * fact, 1.0 / (d + 1));
  }
  for (int k = 0; k < tab->n_modes; ++k) m->dz_lim[k] = m->taylor_thr[kTaylorMax] / m->tau_abs[k];
}

// Benchmark timing state (see fgt_profile_begin).
struct Profiler {
  bool on = false;
  struct Call {
    hipEvent_t ev[kMaxPhases + 1];
    int n;
    bool f64;
  };
  std::vector<Call> calls;
  // Events of earlier sessions, reused so that a session after the first
  // creates none while the calls it times are being enqueued.
  std::vector<hipEvent_t> pool;
  hipError_t take(hipEvent_t* ev) {
    if (!pool.empty()) {
      *ev = pool.back();
      pool.pop_back();
      return hipSuccess;
    }
    return hipEventCreate(ev);
  }
};
static Profiler g_prof;

}  // namespace fgt

struct fgt_plan_s {
  int dtype;
  double delta;
  const fgt::SoeTable* table;
  fgt::Modes modes;
};

namespace fgt {

// fgt_eval of a small problem in one launch (fgt_small.hip), recorded as one
// phase on tl; *done is false, and nothing enqueued or recorded, when the
// problem is too large for it.
template <class T>
hipError_t small_eval(const Workspace& w, const Modes& md, const T* x, int64_t M, const T* y,
                      const T* alpha, int64_t N, T* u, hipStream_t s, Timeline* tl, bool* done);

namespace {

// Sort (when `sort` is set) and evaluate u at the targets.  Small problems run
// in one workgroup (the multi-kernel path is launch-latency bound there).
template <class T>
hipError_t forward(const fgt_plan_s* plan, const Workspace& w, const void* x, int64_t M,
                   const void* y, const void* alpha, int64_t N, void* u, bool sort,
                   hipStream_t s, Timeline* tl) {
  const int64_t P = M + N;
  if (sort) {
    bool done = false;
    const hipError_t e = small_eval<T>(w, plan->modes, (const T*)x, M, (const T*)y,
                                       (const T*)alpha, N, (T*)u, s, tl, &done);
    if (done || e != hipSuccess) return e;
  }
  if (sort) {
    const hipError_t e =
        sort_points<T>(w, (const T*)x, M, (const T*)y, N, plan->modes.sort, s, tl);
    if (e != hipSuccess) return e;
  }
  // The scan's tile reduce gathers alpha into sorted order (ids below N are sources).
  const ScanOut<T> out{(T*)u, nullptr, nullptr, (uint32_t)N, (uint32_t)M};
  return scan_points<T>(w, plan->modes, P, nullptr, (const T*)alpha, (uint32_t)N, out, s, tl);
}

// Gradients of L = sum_i g_i u_i (see fgt_backward): sort if asked, then the
// one adjoint pass over the sorted points.
template <class T>
hipError_t backward(const fgt_plan_s* plan, const Workspace& w, const void* x, int64_t M,
                    const void* y, const void* alpha, int64_t N, const void* g, void* dalpha,
                    void* dx, void* dy, void* ddelta, bool sort, hipStream_t s) {
  if (sort) {
    Timeline none;
    hipError_t e = sort_points<T>(w, (const T*)x, M, (const T*)y, N, plan->modes.sort, s, &none);
    if (e == hipSuccess)
      e = gather_strengths<T>(w, M + N, 0u, (uint32_t)N, (const T*)alpha, (T*)w.b, s);
    if (e != hipSuccess) return e;
  }
  return adjoint_points<T>(w, plan->modes, M, N, (const T*)g, (T*)dx, (T*)dalpha, (T*)dy,
                           (T*)ddelta, plan->delta, s);
}

// Validation and launch of fgt_eval on a given workspace; `profile` records
// the phase events of fgt_profile_begin.
int eval_entry(const fgt_plan_s* plan, const void* x, int64_t M, const void* y, const void* alpha,
               int64_t N, void* u, void* ws, size_t ws_bytes, hipStream_t stream, bool profile) {
  if (!plan || M < 0 || N < 0) return FGT_EINVAL;
  if (M + N >= (int64_t(1) << 32)) return FGT_EINVAL;
  if (M == 0) return FGT_OK;
  if (!x || !u) return FGT_EINVAL;
  const bool f64 = plan->dtype == FGT_F64;
  if (N == 0) {
    hipError_t e = f64 ? fill_zero<double>((double*)u, M, stream)
                       : fill_zero<float>((float*)u, M, stream);
    return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
  }
  if (!y || !alpha || !ws) return FGT_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return FGT_EINVAL;
  const int esz = f64 ? 8 : 4;
  const Workspace w = layout(ws, M + N, esz, plan->modes.n);
  if (ws_bytes < w.total) return FGT_EINVAL;
  Timeline tl;
  Profiler::Call call;
  if (profile) {
    call.n = 0;
    call.f64 = f64;
    for (int i = 0; i <= kMaxPhases; ++i) {
      if (g_prof.take(&call.ev[i]) != hipSuccess) return FGT_EDEVICE;
    }
    tl.ev = call.ev;
    tl.cap = kMaxPhases + 1;
  }
  hipError_t e = f64 ? forward<double>(plan, w, x, M, y, alpha, N, u, true, stream, &tl)
                     : forward<float>(plan, w, x, M, y, alpha, N, u, true, stream, &tl);
  if (profile) {
    call.n = tl.n;
    g_prof.calls.push_back(call);
  }
  return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
}

// Workspace of fgt_eval_noalloc: a fixed device array, one copy per device,
// held until the process ends.  Host code never uses the array's name as a
// device address: the address of each device's copy is taken once, with that
// device current, and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[FGT_NOALLOC_BYTES];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

// The scratch array of the device that `stream` belongs to (the current
// device for the null stream), which must be the current device.
int scratch_of_stream(hipStream_t stream, void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FGT_EDEVICE;
  if (stream) {
    hipDevice_t sdev = -1;
    if (hipStreamGetDevice(stream, &sdev) != hipSuccess) return FGT_EDEVICE;
    if (sdev != dev) return FGT_EINVAL;
  }
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FGT_EDEVICE;
    if (((uintptr_t)p & 255u) != 0) return FGT_EDEVICE;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return FGT_OK;
}

}  // namespace
}  // namespace fgt

extern "C" {

const char* fgt_version(void) { return "fgt-mi355x 0.1 (gfx950)"; }

const char* fgt_strerror(int status) {
  switch (status) {
    case FGT_OK: return "ok";
    case FGT_EINVAL: return "invalid argument";
    case FGT_EUNSUPPORTED: return "unsupported request";
    case FGT_ENONFINITE: return "non-finite coordinate";
    case FGT_EDEVICE: return "HIP runtime error";
    case FGT_EUNSORTED: return "points not in ascending order";
    case FGT_ENOSPACE: return "problem larger than the fixed workspace of fgt_eval_noalloc";
    default: return "unknown status";
  }
}

int fgt_max_digits(int dtype) { return fgt::max_digits(dtype); }

int fgt_plan(double delta, int digits, int dtype, fgt_plan_t* out) {
  if (!out) return FGT_EINVAL;
  *out = nullptr;
  if (!(delta > 0.0) || !isfinite(delta)) return FGT_EINVAL;
  if (dtype != FGT_F64 && dtype != FGT_F32) return FGT_EINVAL;
  if (digits < 1 || digits > fgt::max_digits_f64()) return FGT_EINVAL;
  if (digits > fgt_max_digits(dtype)) return FGT_EUNSUPPORTED;
  const fgt::SoeTable* tab = fgt::choose_table(digits);
  if (!tab) return FGT_EUNSUPPORTED;
  fgt_plan_s* p = new (std::nothrow) fgt_plan_s;
  if (!p) return FGT_EINVAL;
  p->dtype = dtype;
  p->delta = delta;
  p->table = tab;
  fgt::make_modes(tab, delta, dtype, &p->modes);
  *out = p;
  return FGT_OK;
}

int fgt_plan_info(fgt_plan_t plan, int* n_modes, double* err_bound, double* deriv_err_bound,
                  double* tau, double* omega, double* delta) {
  if (!plan) return FGT_EINVAL;
  const int n = plan->modes.n;
  if (n_modes) *n_modes = n;
  if (err_bound) *err_bound = plan->table->err_bound;
  if (deriv_err_bound) *deriv_err_bound = plan->table->deriv_err_bound;
  if (delta) *delta = plan->delta;
  for (int k = 0; k < n; ++k) {
    if (tau) {
      tau[2 * k] = plan->modes.tau_re[k];
      tau[2 * k + 1] = plan->modes.tau_im[k];
    }
    if (omega) {
      omega[2 * k] = plan->modes.om_re[k];
      omega[2 * k + 1] = plan->modes.om_im[k];
    }
  }
  return FGT_OK;
}

void fgt_plan_destroy(fgt_plan_t plan) { delete plan; }

size_t fgt_workspace_size(fgt_plan_t plan, int64_t M, int64_t N) {
  if (!plan || M < 0 || N < 0) return 0;
  const int esz = plan->dtype == FGT_F64 ? 8 : 4;
  return fgt::layout(nullptr, M + N, esz, plan->modes.n).total;
}

int fgt_eval(fgt_plan_t plan, const void* x, int64_t M, const void* y, const void* alpha,
             int64_t N, void* u, void* ws, size_t ws_bytes, hipStream_t stream) {
  return fgt::eval_entry(plan, x, M, y, alpha, N, u, ws, ws_bytes, stream, fgt::g_prof.on);
}

int fgt_eval_noalloc(fgt_plan_t plan, const void* x, int64_t M, const void* y, const void* alpha,
                     int64_t N, void* u, hipStream_t stream) {
  if (!plan || M < 0 || N < 0) return FGT_EINVAL;
  if (M + N >= (int64_t(1) << 32)) return FGT_EINVAL;
  if (fgt_workspace_size(plan, M, N) > (size_t)FGT_NOALLOC_BYTES) return FGT_ENOSPACE;
  if (M == 0) return FGT_OK;
  void* ws = nullptr;
  const int rc = fgt::scratch_of_stream(stream, &ws);
  if (rc != FGT_OK) return rc;
  return fgt::eval_entry(plan, x, M, y, alpha, N, u, ws, (size_t)FGT_NOALLOC_BYTES, stream, false);
}

int fgt_sort(fgt_plan_t plan, const void* x, int64_t M, const void* y, const void* alpha, int64_t N,
             int flags, uint32_t* perm, void* z, double* resolution, void* ws, size_t ws_bytes,
             hipStream_t stream) {
  if (!plan || M < 0 || N < 0) return FGT_EINVAL;
  if (M + N >= (int64_t(1) << 32)) return FGT_EINVAL;
  if (flags & ~FGT_SORT_EXACT) return FGT_EINVAL;
  const bool exact = (flags & FGT_SORT_EXACT) != 0;
  const fgt::SortRes res = exact ? fgt::SortRes{0.0, 0.0, 0.0} : plan->modes.sort;
  if (resolution) {
    resolution[0] = res.key_width;
    resolution[1] = res.code_tol;
  }
  const int64_t P = M + N;
  if (P == 0) return FGT_OK;
  if ((M > 0 && !x) || (N > 0 && !y) || !ws) return FGT_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return FGT_EINVAL;
  const bool f64 = plan->dtype == FGT_F64;
  const fgt::Workspace w = fgt::layout(ws, P, f64 ? 8 : 4, plan->modes.n);
  if (ws_bytes < w.total) return FGT_EINVAL;
  fgt::Timeline none;
  hipError_t e;
  if (f64) {
    e = fgt::sort_points<double>(w, (const double*)x, M, (const double*)y, N, res, stream, &none);
    if (e == hipSuccess && alpha)
      e = fgt::gather_strengths<double>(w, P, 0u, (uint32_t)N, (const double*)alpha,
                                        (double*)w.b, stream);
    if (e == hipSuccess && (perm || z)) e = fgt::copy_sorted<double>(w, P, perm, (double*)z, stream);
  } else {
    e = fgt::sort_points<float>(w, (const float*)x, M, (const float*)y, N, res, stream, &none);
    if (e == hipSuccess && alpha)
      e = fgt::gather_strengths<float>(w, P, 0u, (uint32_t)N, (const float*)alpha, (float*)w.b,
                                       stream);
    if (e == hipSuccess && (perm || z)) e = fgt::copy_sorted<float>(w, P, perm, (float*)z, stream);
  }
  return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
}

int fgt_eval_sorted(fgt_plan_t plan, int64_t M, int64_t N, const void* alpha, void* u, void* ws,
                    size_t ws_bytes, hipStream_t stream) {
  if (!plan || M < 0 || N < 0) return FGT_EINVAL;
  if (M + N >= (int64_t(1) << 32)) return FGT_EINVAL;
  if (M == 0) return FGT_OK;
  if (!u) return FGT_EINVAL;
  const bool f64 = plan->dtype == FGT_F64;
  if (N == 0) {
    hipError_t e = f64 ? fgt::fill_zero<double>((double*)u, M, stream)
                       : fgt::fill_zero<float>((float*)u, M, stream);
    return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
  }
  if (!alpha || !ws) return FGT_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return FGT_EINVAL;
  const fgt::Workspace w = fgt::layout(ws, M + N, f64 ? 8 : 4, plan->modes.n);
  if (ws_bytes < w.total) return FGT_EINVAL;
  fgt::Timeline none;
  hipError_t e = f64 ? fgt::forward<double>(plan, w, nullptr, M, nullptr, alpha, N, u, false, stream, &none)
                     : fgt::forward<float>(plan, w, nullptr, M, nullptr, alpha, N, u, false, stream, &none);
  return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
}

int fgt_eval_self(fgt_plan_t plan, const void* x, int64_t N, const void* alpha, void* u, int flags,
                  void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan || N < 0) return FGT_EINVAL;
  if (N >= (int64_t(1) << 32)) return FGT_EINVAL;
  if (flags & ~FGT_PRESORTED) return FGT_EINVAL;
  if (N == 0) return FGT_OK;
  if (!x || !alpha || !u || !ws) return FGT_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return FGT_EINVAL;
  const bool f64 = plan->dtype == FGT_F64;
  const fgt::Workspace w = fgt::layout(ws, N, f64 ? 8 : 4, plan->modes.n);
  if (ws_bytes < w.total) return FGT_EINVAL;
  fgt::Timeline none;
  hipError_t e;
  // Every point is a source (strength alpha) and a target (output u): merged ids in [0, N).
  if (f64) {
    // Presorted: the strengths are read in place; sorted here: the tile reduce gathers them.
    const bool pre = (flags & FGT_PRESORTED) != 0;
    e = pre ? fgt::presorted_points<double>(w, (const double*)x, (const double*)alpha, N, stream)
            : fgt::sort_points<double>(w, nullptr, 0, (const double*)x, N, plan->modes.sort, stream,
                                       &none);
    if (e == hipSuccess)
      e = fgt::scan_points<double>(w, plan->modes, N, pre ? (const double*)alpha : nullptr,
                                   pre ? nullptr : (const double*)alpha, (uint32_t)N,
                                   fgt::ScanOut<double>{(double*)u, nullptr, nullptr, 0u, (uint32_t)N},
                                   stream, &none);
  } else {
    const bool pre = (flags & FGT_PRESORTED) != 0;
    e = pre ? fgt::presorted_points<float>(w, (const float*)x, (const float*)alpha, N, stream)
            : fgt::sort_points<float>(w, nullptr, 0, (const float*)x, N, plan->modes.sort, stream,
                                      &none);
    if (e == hipSuccess)
      e = fgt::scan_points<float>(w, plan->modes, N, pre ? (const float*)alpha : nullptr,
                                  pre ? nullptr : (const float*)alpha, (uint32_t)N,
                                  fgt::ScanOut<float>{(float*)u, nullptr, nullptr, 0u, (uint32_t)N},
                                  stream, &none);
  }
  return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
}

int fgt_backward(fgt_plan_t plan, const void* x, int64_t M, const void* y, const void* alpha,
                 int64_t N, const void* g, void* dalpha, void* dx, void* dy, void* ddelta,
                 int flags, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan || M < 0 || N < 0) return FGT_EINVAL;
  if (M + N >= (int64_t(1) << 32)) return FGT_EINVAL;
  if (flags & ~FGT_SORTED) return FGT_EINVAL;
  const bool f64 = plan->dtype == FGT_F64;
  auto zero = [&](void* p, int64_t n) -> hipError_t {
    if (!p || n == 0) return hipSuccess;
    return f64 ? fgt::fill_zero<double>((double*)p, n, stream)
               : fgt::fill_zero<float>((float*)p, n, stream);
  };
  if (M == 0 || N == 0) {
    // No pairs: every gradient is zero.
    hipError_t e = zero(dalpha, N);
    if (e == hipSuccess) e = zero(dy, N);
    if (e == hipSuccess) e = zero(dx, M);
    if (e == hipSuccess) e = zero(ddelta, 1);
    return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
  }
  if (!dalpha && !dx && !dy && !ddelta) return FGT_OK;
  const bool sort = !(flags & FGT_SORTED);
  if (!g || !ws || (sort && (!x || !y || !alpha))) return FGT_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return FGT_EINVAL;
  const fgt::Workspace w = fgt::layout(ws, M + N, f64 ? 8 : 4, plan->modes.n);
  if (ws_bytes < w.total) return FGT_EINVAL;
  hipError_t e = f64 ? fgt::backward<double>(plan, w, x, M, y, alpha, N, g, dalpha, dx, dy, ddelta,
                                            sort, stream)
                     : fgt::backward<float>(plan, w, x, M, y, alpha, N, g, dalpha, dx, dy, ddelta,
                                           sort, stream);
  return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
}

}  // extern "C"

struct fgt_batch_s {
  int digits;
  fgt::Modes modes;        // the table at delta = 1
  double s_allow;          // sort resolution in scaled coordinates
  fgt::BatchDims dims;     // sizes for the workspace: maxima over the tunable choices
  // Device tables for the two bucket sizes the autotuner chooses between.
  fgt::SegInfo* d_seg[2];
  fgt::BucketInfo* d_buckets[2];
  int64_t n_buckets[2];
  int max_nb_log2[2];
  fgt::ChunkInfo* d_chunks;
  int64_t* d_ne_base;
  double* d_ne_scale;
  int chunk;               // points per lane in the scan: 8 or 16
  int bucket_sel;          // 0: buckets of about 2048 points, 1: about 1024
};

namespace fgt {
namespace {

constexpr int kBucketTargets[2] = {2048, 1024};
constexpr int kChunkChoices[2] = {16, 8};

void batch_free(fgt_batch_s* b) {
  if (!b) return;
  for (int i = 0; i < 2; ++i) {
    if (b->d_seg[i]) (void)hipFree(b->d_seg[i]);
    if (b->d_buckets[i]) (void)hipFree(b->d_buckets[i]);
  }
  if (b->d_chunks) (void)hipFree(b->d_chunks);
  if (b->d_ne_base) (void)hipFree(b->d_ne_base);
  if (b->d_ne_scale) (void)hipFree(b->d_ne_scale);
  delete b;
}

// Host part of a batch plan for one bucket size: validation, per-transform
// tables, sizes.
int batch_tables(int64_t B, const double* delta, const int64_t* x_off, const int64_t* y_off, int R,
                 int bucket_target, std::vector<SegInfo>& seg, std::vector<ChunkInfo>& chunks,
                 std::vector<BucketInfo>& buckets, std::vector<int64_t>& ne_base,
                 std::vector<double>& ne_scale, BatchDims& d, int& max_nb_log2) {
  if (B < 0 || R < 1 || R > 64) return FGT_EINVAL;
  if (B > 0 && (!delta || !x_off || !y_off)) return FGT_EINVAL;
  if (B > (int64_t(1) << 30)) return FGT_EINVAL;
  if (B > 0 && (x_off[0] != 0 || y_off[0] != 0)) return FGT_EINVAL;
  memset(&d, 0, sizeof(d));
  seg.clear();
  chunks.clear();
  buckets.clear();
  ne_base.clear();
  ne_scale.clear();
  d.B = B;
  d.R = R;
  max_nb_log2 = 0;
  int64_t base = 0, chunk0 = 0, bucket0 = 0, cnt0 = 0;
  seg.resize((size_t)B);
  for (int64_t b = 0; b < B; ++b) {
    const int64_t M = x_off[b + 1] - x_off[b];
    const int64_t N = y_off[b + 1] - y_off[b];
    if (M < 0 || N < 0) return FGT_EINVAL;
    if (!(delta[b] > 0.0) || !isfinite(delta[b])) return FGT_EINVAL;
    const int64_t Pb = M + N;
    SegInfo& sg = seg[(size_t)b];
    sg.x_off = x_off[b];
    sg.y_off = y_off[b];
    sg.M = M;
    sg.N = N;
    sg.base = base;
    sg.scale = 1.0 / sqrt(delta[b]);
    if (!isfinite(sg.scale)) return FGT_EINVAL;
    sg.n_chunks = (int32_t)((Pb + kBChunk - 1) / kBChunk);
    int lg = 0;
    while (lg < kMaxBucketLog2 && ((int64_t)bucket_target << lg) < Pb) ++lg;
    sg.nb_log2 = lg;
    if (lg > max_nb_log2) max_nb_log2 = lg;
    sg.chunk0 = chunk0;
    sg.bucket0 = bucket0;
    sg.cnt0 = cnt0;
    for (int32_t c = 0; c < sg.n_chunks; ++c) chunks.push_back(ChunkInfo{(int32_t)b, 0, (int64_t)c * kBChunk});
    for (int32_t k = 0; k < (1 << lg); ++k) buckets.push_back(BucketInfo{(int32_t)b, k});
    chunk0 += sg.n_chunks;
    bucket0 += 1 << lg;
    cnt0 += (int64_t)(1 << lg) * sg.n_chunks;
    if (Pb > 0) {
      ne_base.push_back(base);
      ne_scale.push_back(sg.scale);
    }
    base += Pb;
  }
  d.SN = B > 0 ? y_off[B] : 0;
  d.SM = B > 0 ? x_off[B] : 0;
  d.P = base;
  if (d.SN + d.SM > (int64_t)0x7ffffffe) return FGT_EINVAL;
  d.n_chunks = chunk0;
  d.n_buckets = bucket0;
  d.n_counts = cnt0;
  d.K = (int64_t)ne_base.size();
  d.tiles = (d.P + kBTileMin - 1) / kBTileMin;   // the most tiles any chunk choice uses
  if (d.tiles < 1) d.tiles = 1;
  return FGT_OK;
}

// Workspace sizes covering both bucket sizes.
int batch_dims(int64_t B, const double* delta, const int64_t* x_off, const int64_t* y_off, int R,
               int n_modes, BatchDims& d) {
  std::vector<SegInfo> seg;
  std::vector<ChunkInfo> chunks;
  std::vector<BucketInfo> buckets;
  std::vector<int64_t> ne_base;
  std::vector<double> ne_scale;
  BatchDims d1;
  int lg = 0;
  int rc = batch_tables(B, delta, x_off, y_off, R, kBucketTargets[0], seg, chunks, buckets, ne_base,
                        ne_scale, d, lg);
  if (rc != FGT_OK) return rc;
  rc = batch_tables(B, delta, x_off, y_off, R, kBucketTargets[1], seg, chunks, buckets, ne_base,
                    ne_scale, d1, lg);
  if (rc != FGT_OK) return rc;
  if (d1.n_buckets > d.n_buckets) d.n_buckets = d1.n_buckets;
  if (d1.n_counts > d.n_counts) d.n_counts = d1.n_counts;
  d.n_modes = n_modes;
  return FGT_OK;
}

template <class V>
hipError_t upload(const std::vector<V>& v, V** out) {
  *out = nullptr;
  const size_t bytes = sizeof(V) * (v.empty() ? 1 : v.size());
  hipError_t e = hipMalloc((void**)out, bytes);
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*out, v.data(), sizeof(V) * v.size(), hipMemcpyHostToDevice);
  return e;
}

BatchTables tables_of(const fgt_batch_s* b) {
  const int i = b->bucket_sel;
  return BatchTables{b->d_seg[i], b->d_chunks, b->d_buckets[i], b->d_ne_base, b->d_ne_scale,
                     b->n_buckets[i], b->max_nb_log2[i]};
}

// Shape signature of a batch for the tuning cache.
void batch_signature(const fgt_batch_s* b, char* out, size_t n) {
  int lgP = 0;
  while (lgP < 62 && (int64_t(1) << lgP) < b->dims.P) ++lgP;
  int lgB = 0;
  while (lgB < 62 && (int64_t(1) << lgB) < b->dims.B) ++lgB;
  snprintf(out, n, "gfx950:B2^%d:P2^%d:R%d:modes%d", lgB, lgP, b->dims.R, b->modes.n);
}

// Reads "<sig>": {"chunk": c, "bucket": k ...} from a cache file written by
// fgt_batch_tune.  Returns true if found.
bool cache_lookup(const char* path, const char* sig, int* chunk, int* bucket) {
  FILE* f = fopen(path, "rb");
  if (!f) return false;
  std::vector<char> buf;
  char tmp[4096];
  size_t got;
  while ((got = fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + got);
  fclose(f);
  buf.push_back('\0');
  std::string key = std::string("\"") + sig + "\"";
  const char* at = strstr(buf.data(), key.c_str());
  if (!at) return false;
  const char* c = strstr(at, "\"chunk\":");
  const char* k = strstr(at, "\"bucket\":");
  const char* end = strchr(at, '}');
  if (!c || !k || !end || c > end || k > end) return false;
  const int cv = atoi(c + 8), kv = atoi(k + 9);
  if ((cv != 8 && cv != 16) || (kv != 1024 && kv != 2048)) return false;
  *chunk = cv;
  *bucket = kv;
  return true;
}

// Rewrites the cache file with this signature's entry replaced or added.
void cache_store(const char* path, const char* sig, int chunk, int bucket, const double* ms,
                 int n_candidates) {
  std::vector<std::string> lines;
  if (FILE* f = fopen(path, "rb")) {
    char line[4096];
    while (fgets(line, sizeof(line), f)) {
      std::string l(line);
      if (l.find("\"gfx950:") != std::string::npos && l.find(std::string("\"") + sig + "\"") == std::string::npos)
        lines.push_back(l.substr(0, l.find_last_not_of(",\n\r ") + 1));
    }
    fclose(f);
  }
  char entry[1024];
  int off = snprintf(entry, sizeof(entry), "  \"%s\": {\"chunk\": %d, \"bucket\": %d, \"ms\": [", sig,
                     chunk, bucket);
  for (int i = 0; i < n_candidates && off < (int)sizeof(entry) - 32; ++i)
    off += snprintf(entry + off, sizeof(entry) - off, "%s%.4f", i ? ", " : "", ms[i]);
  snprintf(entry + off, sizeof(entry) - off, "]}");
  lines.push_back(entry);
  std::string tmp_path = std::string(path) + ".tmp";
  FILE* f = fopen(tmp_path.c_str(), "wb");
  if (!f) return;
  fputs("{\n", f);
  for (size_t i = 0; i < lines.size(); ++i) {
    fputs(lines[i].c_str(), f);
    fputs(i + 1 < lines.size() ? ",\n" : "\n", f);
  }
  fputs("}\n", f);
  fclose(f);
  (void)rename(tmp_path.c_str(), path);
}

}  // namespace
}  // namespace fgt

extern "C" {

int fgt_batch_plan(int64_t B, const double* delta, int digits, int dtype, const int64_t* x_off,
                   const int64_t* y_off, int R, fgt_batch_t* out) {
  if (!out) return FGT_EINVAL;
  *out = nullptr;
  if (dtype != FGT_F64 && dtype != FGT_F32) return FGT_EINVAL;
  if (digits < 1 || digits > fgt::max_digits_f64()) return FGT_EINVAL;
  if (dtype != FGT_F64) return FGT_EUNSUPPORTED;
  const fgt::SoeTable* tab = fgt::choose_table(digits);
  if (!tab) return FGT_EUNSUPPORTED;
  fgt::BatchDims d;
  int rc = fgt::batch_dims(B, delta, x_off, y_off, R, tab->n_modes, d);
  if (rc != FGT_OK) return rc;
  fgt_batch_s* b = new (std::nothrow) fgt_batch_s;
  if (!b) return FGT_EINVAL;
  memset(b, 0, sizeof(*b));
  b->digits = digits;
  fgt::make_modes(tab, 1.0, FGT_F64, &b->modes);
  b->s_allow = b->modes.key_width;
  b->dims = d;
  b->chunk = fgt::kChunkChoices[0];
  b->bucket_sel = 0;
  for (int i = 0; i < 2; ++i) {
    std::vector<fgt::SegInfo> seg;
    std::vector<fgt::ChunkInfo> chunks;
    std::vector<fgt::BucketInfo> buckets;
    std::vector<int64_t> ne_base;
    std::vector<double> ne_scale;
    fgt::BatchDims di;
    int lg = 0;
    (void)fgt::batch_tables(B, delta, x_off, y_off, R, fgt::kBucketTargets[i], seg, chunks, buckets,
                            ne_base, ne_scale, di, lg);
    b->n_buckets[i] = di.n_buckets;
    b->max_nb_log2[i] = lg;
    bool ok = fgt::upload(seg, &b->d_seg[i]) == hipSuccess &&
              fgt::upload(buckets, &b->d_buckets[i]) == hipSuccess;
    if (ok && i == 0)
      ok = fgt::upload(chunks, &b->d_chunks) == hipSuccess &&
           fgt::upload(ne_base, &b->d_ne_base) == hipSuccess &&
           fgt::upload(ne_scale, &b->d_ne_scale) == hipSuccess;
    if (!ok) {
      fgt::batch_free(b);
      return FGT_EDEVICE;
    }
  }
  *out = b;
  return FGT_OK;
}

size_t fgt_batch_workspace_size(fgt_batch_t plan) {
  if (!plan) return 0;
  return fgt::batch_layout(nullptr, plan->dims).total;
}

int fgt_batch_info(fgt_batch_t plan, int* n_modes, double* err_bound, int64_t* total_points) {
  if (!plan) return FGT_EINVAL;
  if (n_modes) *n_modes = plan->modes.n;
  if (err_bound) *err_bound = fgt::choose_table(plan->digits)->err_bound;
  if (total_points) *total_points = plan->dims.P;
  return FGT_OK;
}

int fgt_batch_config(fgt_batch_t plan, int* chunk, int* bucket_points) {
  if (!plan) return FGT_EINVAL;
  if (chunk) *chunk = plan->chunk;
  if (bucket_points) *bucket_points = fgt::kBucketTargets[plan->bucket_sel];
  return FGT_OK;
}

int fgt_batch_set_config(fgt_batch_t plan, int chunk, int bucket_points) {
  if (!plan) return FGT_EINVAL;
  if (chunk != 8 && chunk != 16) return FGT_EINVAL;
  if (bucket_points != fgt::kBucketTargets[0] && bucket_points != fgt::kBucketTargets[1])
    return FGT_EINVAL;
  plan->chunk = chunk;
  plan->bucket_sel = bucket_points == fgt::kBucketTargets[0] ? 0 : 1;
  return FGT_OK;
}

int fgt_batch_eval(fgt_batch_t plan, const void* x, const void* y, const void* alpha, void* u,
                   void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan) return FGT_EINVAL;
  const fgt::BatchDims& d = plan->dims;
  if ((d.SM > 0 && (!x || !u)) || (d.SN > 0 && (!y || !alpha)) || !ws) return FGT_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return FGT_EINVAL;
  const fgt::BatchWork w = fgt::batch_layout(ws, d);
  if (ws_bytes < w.total) return FGT_EINVAL;
  hipError_t e = fgt::batch_eval_launch(d, fgt::tables_of(plan), plan->modes, plan->s_allow,
                                        plan->chunk, (const double*)x, (const double*)y,
                                        (const double*)alpha, (double*)u, w, stream);
  return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
}

int fgt_batch_sorted(fgt_batch_t plan, const void* ws, size_t ws_bytes, uint32_t* codes, void* z,
                     double* resolution, hipStream_t stream) {
  if (!plan || !ws) return FGT_EINVAL;
  if (((uintptr_t)ws & 255u) != 0) return FGT_EINVAL;
  const fgt::BatchWork w = fgt::batch_layout(const_cast<void*>(ws), plan->dims);
  if (ws_bytes < w.total) return FGT_EINVAL;
  if (resolution) *resolution = plan->s_allow;
  const hipError_t e = fgt::batch_sorted_copy(plan->dims, w, codes, (double*)z, stream);
  return e == hipSuccess ? FGT_OK : FGT_EDEVICE;
}

int fgt_batch_tune(fgt_batch_t plan, const void* x, const void* y, const void* alpha, void* u,
                   void* ws, size_t ws_bytes, hipStream_t stream, const char* cache_path) {
  if (!plan) return FGT_EINVAL;
  char sig[160];
  fgt::batch_signature(plan, sig, sizeof(sig));
  int chunk = 0, bucket = 0;
  if (cache_path && fgt::cache_lookup(cache_path, sig, &chunk, &bucket))
    return fgt_batch_set_config(plan, chunk, bucket);
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess) return FGT_EDEVICE;
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return FGT_EDEVICE;
  }
  double ms[4];
  int best = -1;
  int rc = FGT_OK;
  for (int c = 0; c < 4 && rc == FGT_OK; ++c) {
    rc = fgt_batch_set_config(plan, fgt::kChunkChoices[c % 2], fgt::kBucketTargets[c / 2]);
    if (rc == FGT_OK) rc = fgt_batch_eval(plan, x, y, alpha, u, ws, ws_bytes, stream);   // warm-up
    if (rc != FGT_OK) break;
    if (hipEventRecord(ev[0], stream) != hipSuccess) rc = FGT_EDEVICE;
    for (int r = 0; r < 3 && rc == FGT_OK; ++r)
      rc = fgt_batch_eval(plan, x, y, alpha, u, ws, ws_bytes, stream);
    float t = 0.f;
    if (rc == FGT_OK && (hipEventRecord(ev[1], stream) != hipSuccess ||
                         hipEventSynchronize(ev[1]) != hipSuccess ||
                         hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess))
      rc = FGT_EDEVICE;
    ms[c] = t / 3.0;
    if (rc == FGT_OK && (best < 0 || ms[c] < ms[best])) best = c;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (rc != FGT_OK || best < 0) return rc != FGT_OK ? rc : FGT_EDEVICE;
  rc = fgt_batch_set_config(plan, fgt::kChunkChoices[best % 2], fgt::kBucketTargets[best / 2]);
  if (rc == FGT_OK && cache_path)
    fgt::cache_store(cache_path, sig, fgt::kChunkChoices[best % 2], fgt::kBucketTargets[best / 2],
                     ms, 4);
  return rc;
}

void fgt_batch_destroy(fgt_batch_t plan) { fgt::batch_free(plan); }

size_t fgt_eval_batched_workspace_size(int64_t B, const int64_t* x_off, const int64_t* y_off, int R,
                                       int digits) {
  const fgt::SoeTable* tab = (digits >= 1 && digits <= fgt::max_digits_f64()) ? fgt::choose_table(digits) : nullptr;
  if (!tab || B < 0 || (B > 0 && (!x_off || !y_off))) return 0;
  std::vector<double> ones((size_t)(B > 0 ? B : 1), 1.0);
  fgt::BatchDims d;
  if (fgt::batch_dims(B, ones.data(), x_off, y_off, R, tab->n_modes, d) != FGT_OK) return 0;
  return fgt::batch_layout(nullptr, d).total;
}

int fgt_eval_batched(int64_t B, const double* delta, int digits, int dtype, const int64_t* x_off,
                     const int64_t* y_off, const void* x, const void* y, const void* alpha, int R,
                     void* u, void* ws, size_t ws_bytes, hipStream_t stream) {
  fgt_batch_t plan = nullptr;
  int rc = fgt_batch_plan(B, delta, digits, dtype, x_off, y_off, R, &plan);
  if (rc != FGT_OK) return rc;
  rc = fgt_batch_eval(plan, x, y, alpha, u, ws, ws_bytes, stream);
  // The plan's tables are in use by the enqueued kernels until the stream drains.
  if (hipStreamSynchronize(stream) != hipSuccess && rc == FGT_OK) rc = FGT_EDEVICE;
  fgt_batch_destroy(plan);
  return rc;
}

int fgt_profile_begin(void) {
  fgt::g_prof.on = true;
  return FGT_OK;
}

static const char* const kPhaseNamesF64[] = {"setup", "radix0", "radix1", "radix2", "radix3",
                                             "radix4", "radix5", "radix6", "radix7",
                                             "tiles_reduce", "carry", "tiles_final"};

const char* fgt_profile_phase_name(int phase) {
  if (phase < 0 || phase >= fgt::kMaxPhases) return "";
  return kPhaseNamesF64[phase];
}

int fgt_profile_end(double* ms, int max_phases, int* n_phases, int* n_calls) {
  fgt::g_prof.on = false;
  double acc[fgt::kMaxPhases] = {0};
  int phases = 0;
  int rc = FGT_OK;
  for (auto& c : fgt::g_prof.calls) {
    // FP32 has 4 radix passes: map its phases onto the FP64 names.
    const int passes = c.f64 ? 8 : 4;
    // More marks than events: reported as more phases than there are names.
    if (c.n > fgt::kMaxPhases + 1 && c.n - 1 > phases) phases = c.n - 1;
    const int recorded = c.n < fgt::kMaxPhases + 1 ? c.n : fgt::kMaxPhases + 1;
    for (int i = 0; i + 1 < recorded; ++i) {
      float t = 0.f;
      if (hipEventSynchronize(c.ev[i + 1]) != hipSuccess ||
          hipEventElapsedTime(&t, c.ev[i], c.ev[i + 1]) != hipSuccess) {
        rc = FGT_EDEVICE;
        continue;
      }
      const int name = i <= passes ? i : i + (8 - passes);
      if (name >= fgt::kMaxPhases) continue;
      acc[name] += t;
      if (name + 1 > phases) phases = name + 1;
    }
    for (int i = 0; i <= fgt::kMaxPhases; ++i) fgt::g_prof.pool.push_back(c.ev[i]);
  }
  if (n_calls) *n_calls = (int)fgt::g_prof.calls.size();
  fgt::g_prof.calls.clear();
  if (n_phases) *n_phases = phases;
  if (ms)
    for (int i = 0; i < max_phases && i < fgt::kMaxPhases; ++i) ms[i] = acc[i];
  return rc;
}

int fgt_last_device_status(void* ws, hipStream_t stream) {
  if (!ws) return FGT_EINVAL;
  // The status word sits at offset 0 of every layout.
  uint32_t* status = (uint32_t*)ws;
  uint32_t v = 0;
  if (hipStreamSynchronize(stream) != hipSuccess) return FGT_EDEVICE;
  if (hipMemcpy(&v, status, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return FGT_EDEVICE;
  const uint32_t zero = 0;
  if (hipMemcpy(status, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
    return FGT_EDEVICE;
  if (v & fgt::kStatusNonFinite) return FGT_ENONFINITE;
  if (v & fgt::kStatusUnsorted) return FGT_EUNSORTED;
  return v ? FGT_EDEVICE : FGT_OK;
}

}  // extern "C"
