/*
 * orc_real.h -- scalar type of the oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The plain build uses `real` = double.  The counting build (-DORC_COUNT)
 * replaces it by a class that performs the same binary64 arithmetic and
 * counts each operation, so that the algorithmic operation count per
 * cell-update comes from the very code that defines the method.
 * The nudged build (-DORC_NUDGE) moves every transcendental result by one
 * ulp; with multiply-add contraction it gives a second valid rounding of
 * the whole computation, used to measure each cell's conditioning.
 * Operations with an exact-zero operand are not counted: they are the
 * structural zeros of the sparse derivative bookkeeping (for example the
 * y-partials of a temperature-only rate coefficient), which an implementation
 * that tracks sparsity never executes.
 */
#ifndef ORC_REAL_H
#define ORC_REAL_H
#include <cmath>

#ifndef ORC_COUNT

typedef double real;
#if defined(ORC_NUDGE)
/* Conditioning probe: every transcendental result moved by one unit in the
 * last place (up, or down with ORC_NUDGE_DOWN) -- what another faithfully
 * rounded math library may return.  Only used to measure how far rounding
 * alone moves a result. */
#ifdef ORC_NUDGE_DOWN
static inline real nudge(real v) { return std::nextafter(v, -HUGE_VAL); }
#else
static inline real nudge(real v) { return std::nextafter(v, HUGE_VAL); }
#endif
#else
static inline real nudge(real v) { return v; }
#endif
static inline real rexp(real x) { return nudge(std::exp(x)); }
static inline real rlog(real x) { return nudge(std::log(x)); }
static inline real rlog1p(real x) { return nudge(std::log1p(x)); }
#ifdef ORC_NUDGE_DOWN
/* the same probe also forms powers as exp(y log x), whose rounding error
 * grows with |y log x| */
static inline real rpow(real x, real y) { return nudge(std::exp(y * std::log(x))); }
#else
static inline real rpow(real x, real y) { return nudge(std::pow(x, y)); }
#endif
static inline real rsqrt(real x) { return std::sqrt(x); }
static inline double rval(real x) { return x; }

#else

struct OrcCounts {
  double add, mul, div, sqrt_, transc, cmp;
};
extern thread_local OrcCounts orc_counts;

struct CReal {
  double v;
  CReal() : v(0.0) {}
  CReal(double x) : v(x) {}
};
typedef CReal real;

static inline bool nz(const CReal& a) { return a.v != 0.0; }
static inline CReal operator+(CReal a, CReal b) {
  if (nz(a) && nz(b)) orc_counts.add += 1;
  return CReal(a.v + b.v);
}
static inline CReal operator-(CReal a, CReal b) {
  if (nz(a) && nz(b)) orc_counts.add += 1;
  return CReal(a.v - b.v);
}
static inline CReal operator-(CReal a) { return CReal(-a.v); }
static inline CReal operator*(CReal a, CReal b) {
  if (nz(a) && nz(b)) orc_counts.mul += 1;
  return CReal(a.v * b.v);
}
static inline CReal operator/(CReal a, CReal b) {
  if (nz(a)) orc_counts.div += 1;
  return CReal(a.v / b.v);
}
static inline CReal& operator+=(CReal& a, CReal b) { a = a + b; return a; }
static inline CReal& operator-=(CReal& a, CReal b) { a = a - b; return a; }
static inline CReal& operator*=(CReal& a, CReal b) { a = a * b; return a; }
static inline CReal& operator/=(CReal& a, CReal b) { a = a / b; return a; }
#define ORC_CMP(op)                                                   \
  static inline bool operator op(CReal a, CReal b) {                  \
    orc_counts.cmp += 1;                                              \
    return a.v op b.v;                                                \
  }
ORC_CMP(<) ORC_CMP(>) ORC_CMP(<=) ORC_CMP(>=) ORC_CMP(==) ORC_CMP(!=)
#undef ORC_CMP
static inline CReal rexp(CReal x) { orc_counts.transc += 1; return CReal(std::exp(x.v)); }
static inline CReal rlog(CReal x) { orc_counts.transc += 1; return CReal(std::log(x.v)); }
static inline CReal rlog1p(CReal x) { orc_counts.transc += 1; return CReal(std::log1p(x.v)); }
static inline CReal rpow(CReal x, CReal y) { orc_counts.transc += 1; return CReal(std::pow(x.v, y.v)); }
static inline CReal rsqrt(CReal x) { orc_counts.sqrt_ += 1; return CReal(std::sqrt(x.v)); }
static inline double rval(CReal x) { return x.v; }

#endif

static inline real rabs(real x) { return x < real(0.0) ? -x : x; }
static inline real rmax(real a, real b) { return a < b ? b : a; }
static inline real rmin(real a, real b) { return b < a ? b : a; }

#endif
