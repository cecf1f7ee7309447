// CPU check of the FP64 sort-key code of the library (Codec<double>,
// make_codec in csrc/fgt_internal.h), compiled for the host only.
//
// For point sets of many kinds of range it checks what the sort and the scans
// rely on: keys of the grid code stay below 2^63; the key order never
// contradicts the coordinate order; coordinates on the grid decode exactly and
// the others move by less than the grid step g; neighbours differ by less than
// (key difference + 1) g, the bound the sort's resolution rule uses; the grid
// code is taken without any tolerance when every point lies on the grid (the
// data's granularity), and IEEE order keys where the range is degenerate or an
// off-grid shift would exceed the tolerance, and they decode exactly.  Prints one line per case (and one
// per failed check) and exits non-zero if any check failed.
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <vector>

#include "../paper_1909_09825_amd/csrc/fgt_internal.h"

using fgt::Codec;
using fgt::from_key;
using fgt::granularity_exp;
using fgt::make_codec;
using fgt::to_key;

namespace {

struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uni() { return (double)(next() >> 11) * 0x1p-53; }   // [0, 1), 53 random bits
};

int failures = 0;

void fail(const char* name, const char* what, double z) {
  printf("FAIL %s: %s (z = %.17g)\n", name, what, z);
  ++failures;
}

// expect: 1 grid code, 0 IEEE keys, -1 either.
void check(const char* name, const std::vector<double>& z, double tol, int expect) {
  uint64_t kmin = ~0ull, kmax = 0ull;
  int gran = 1 << 20;
  for (double v : z) {
    kmin = std::min(kmin, to_key(v));
    kmax = std::max(kmax, to_key(v));
    if (v != 0.0 && isfinite(v)) gran = std::min(gran, granularity_exp(v));
  }
  const Codec<double> c = make_codec(kmin, kmax, gran, tol);
  if (expect >= 0 && c.quant != expect) {
    fail(name, expect ? "expected the grid code" : "expected IEEE keys", 0.0);
    return;
  }
  const double small = c.quant ? ldexp(c.g, 52) : 0.0;   // below it a point may be off the grid
  std::vector<uint64_t> q(z.size());
  double max_off = 0.0;
  for (size_t i = 0; i < z.size(); ++i) {
    q[i] = c.encode(z[i]);
    const double d = c.decode(q[i]);
    if (!c.quant) {
      if (!(d == z[i]) && !(isnan(d) && isnan(z[i]))) fail(name, "IEEE key does not decode exactly", z[i]);
      continue;
    }
    if (q[i] >= (uint64_t(1) << 63)) fail(name, "key not below 2^63", z[i]);
    if (c.L != 0.0 || fabs(z[i]) >= small) {
      if (d != z[i]) fail(name, "grid point does not decode exactly", z[i]);
    } else {
      const double off = fabs(d - z[i]);
      max_off = std::max(max_off, off);
      if (!(off < c.g)) fail(name, "off-grid point moved by g or more", z[i]);
      if (off > tol) fail(name, "point moved by more than the tolerance", z[i]);
    }
  }
  bool any_nan = false;
  for (double v : z) any_nan |= isnan(v) != 0;
  if (any_nan) {
    printf("ok   %-28s n=%-7zu IEEE          (order not checked: NaN)\n", name, z.size());
    return;
  }
  std::vector<size_t> idx(z.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return z[a] < z[b]; });
  for (size_t j = 1; j < idx.size(); ++j) {
    const double za = z[idx[j - 1]], zb = z[idx[j]];
    const uint64_t qa = q[idx[j - 1]], qb = q[idx[j]];
    if (c.quant ? qb < qa : to_key(zb) < to_key(za)) fail(name, "key order contradicts coordinates", zb);
    // The sort's resolution rule needs this for keys that agree in their high
    // digits; beyond 2^52 key steps it is not checkable in FP64 (and not needed).
    if (c.quant && qb - qa < (uint64_t(1) << 52) &&
        !(zb - za < ((double)(qb - qa) + 1.0) * c.g))
      fail(name, "gap above (dq + 1) g", zb);
  }
  printf("ok   %-28s n=%-7zu %s g=%.3g off-grid max shift %.3g\n", name, z.size(),
         c.quant ? (c.L != 0.0 ? "grid (offset)" : "grid (fixed) ") : "IEEE         ", c.g, max_off);
}

}  // namespace

int main() {
  SplitMix r{1909};
  const int n = 100000;
  std::vector<double> z;

  z.clear();
  for (int i = 0; i < n; ++i) z.push_back(r.uni());
  check("uniform [0,1)", z, 1e-15, 1);
  check("uniform [0,1), no tolerance", z, 0.0, 1);   // multiples of 2^-53: all on the grid

  z.clear();
  for (int i = 0; i < n; ++i) z.push_back(r.uni() / 3.0);
  check("[0,1/3), full significands", z, 1e-15, 1);
  check("[0,1/3), tight tol", z, 1e-30, 0);

  z.clear();
  for (int i = 0; i < n; ++i) z.push_back(r.uni());
  for (double t : {1e-20, 3e-310, 0.0, -0.0, 0x1p-70, 1.5e-9, 0x1p-9 + 0x1p-60}) z.push_back(t);
  check("[0,1) with tiny values", z, 1e-15, 1);
  check("[0,1) tiny values, tight tol", z, 1e-30, 0);

  z.clear();
  for (int i = 0; i < n; ++i) z.push_back(1e6 + r.uni());
  check("[1e6, 1e6+1)", z, 0.0, 1);

  z.clear();
  for (int i = 0; i < n; ++i) z.push_back(-5e3 - 2.0 * r.uni());
  check("[-5002, -5000)", z, 0.0, 1);

  z.clear();
  for (int i = 0; i < n; ++i) z.push_back(-1e6 + 2e6 * r.uni());
  check("[-1e6, 1e6), loose tol", z, 1e-9, 1);
  check("[-1e6, 1e6), all on grid", z, 0.0, 1);
  z.push_back(1e-300);
  check("[-1e6, 1e6) + 1e-300", z, 1e-20, 0);

  z.clear();
  for (int i = 0; i < n; ++i) z.push_back(5.0 + 2.0 * r.uni());
  check("[5, 7)", z, 0.0, 1);

  z.clear();
  for (int i = 0; i < n; ++i) z.push_back(-1.0 + 2.0 * r.uni());
  check("[-1, 1)", z, 1e-15, 1);

  z.assign(1000, 0.3);
  check("all equal", z, 1.0, 0);

  z = {0.25, 0.75, 0.5};
  check("three points", z, 0.0, 1);

  z.clear();
  for (int i = 0; i < n; ++i) {
    const double m = pow(10.0, -10.0 + 20.0 * r.uni());
    z.push_back((r.next() & 1) ? m : -m);
  }
  check("log-uniform 1e-10..1e10 +-", z, 1.0, 1);

  z.clear();
  for (int i = 0; i < n; ++i) z.push_back(-1e300 + 2e300 * r.uni());
  check("[-1e300, 1e300)", z, 1e300, 1);

  z = {-1.7e308, 1.7e308, 0.0, 1.0};
  check("range overflows", z, 1e300, 0);

  z = {1e-310, 2e-310, 1.5e-310};
  check("subnormal range", z, 1.0, 0);

  z = {0.1, NAN, 0.2};
  check("with NaN", z, 1.0, 0);

  z = {0.1, INFINITY, 0.2};
  check("with infinity", z, 1.0, 0);

  if (failures) {
    printf("%d failures\n", failures);
    return 1;
  }
  printf("all cases passed\n");
  return 0;
}
