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
 * The reciprocal build (-DORC_RCP) forms every quotient a / b as a times a
 * rounded reciprocal of b (moved by one ulp up, or down with
 * ORC_NUDGE_DOWN), the rounding class of an implementation that divides
 * through a hardware reciprocal estimate refined by Newton steps; it too
 * only measures conditioning.  With ORC_NUDGE as well (and multiply-add
 * contraction) it moves every rounding class at once, as an implementation
 * with its own elementary functions and division does.
 * Operations with an exact-zero operand are not counted: they are the
 * structural zeros of the sparse derivative bookkeeping (for example the
 * y-partials of a temperature-only rate coefficient), which an implementation
 * that tracks sparsity never executes.
 */
#ifndef ORC_REAL_H
#define ORC_REAL_H
#include <cmath>

#if !defined(ORC_COUNT) && !defined(ORC_RCP)

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
#ifdef ORC_COEF32
/* Binary32 probe: every exponential and power (the rate, cooling and
 * opacity coefficients are built from them) rounded to binary32, the rest
 * of the arithmetic binary64.  It measures how far coefficients of binary32
 * accuracy alone move a cell's result, the error floor of any mixed
 * binary32 / binary64 implementation. */
static inline real rexp(real x) { return double(float(std::exp(x))); }
#else
static inline real rexp(real x) { return nudge(std::exp(x)); }
#endif
static inline real rlog(real x) { return nudge(std::log(x)); }
static inline real rlog1p(real x) { return nudge(std::log1p(x)); }
#ifdef ORC_NUDGE_DOWN
/* the same probe also forms powers as exp(y log x), whose rounding error
 * grows with |y log x| */
static inline real rpow(real x, real y) { return nudge(std::exp(y * std::log(x))); }
#elif defined(ORC_COEF32)
static inline real rpow(real x, real y) { return double(float(std::pow(x, y))); }
#else
static inline real rpow(real x, real y) { return nudge(std::pow(x, y)); }
#endif
static inline real rsqrt(real x) { return std::sqrt(x); }
static inline double rval(real x) { return x; }

#else

#ifdef ORC_COUNT
struct OrcCounts {
  double add, mul, div, sqrt_, transc, cmp;
};
extern thread_local OrcCounts orc_counts;
#define ORC_TALLY(field) (orc_counts.field += 1)
#else
#define ORC_TALLY(field) ((void)0)
#endif

struct CReal {
  double v;
  CReal() : v(0.0) {}
  CReal(double x) : v(x) {}
};
typedef CReal real;

static inline bool nz(const CReal& a) { return a.v != 0.0; }
static inline CReal operator+(CReal a, CReal b) {
  if (nz(a) && nz(b)) ORC_TALLY(add);
  return CReal(a.v + b.v);
}
static inline CReal operator-(CReal a, CReal b) {
  if (nz(a) && nz(b)) ORC_TALLY(add);
  return CReal(a.v - b.v);
}
static inline CReal operator-(CReal a) { return CReal(-a.v); }
static inline CReal operator*(CReal a, CReal b) {
  if (nz(a) && nz(b)) ORC_TALLY(mul);
  return CReal(a.v * b.v);
}
static inline CReal operator/(CReal a, CReal b) {
  if (nz(a)) ORC_TALLY(div);
#ifdef ORC_RCP
#ifdef ORC_NUDGE_DOWN
  return CReal(a.v * std::nextafter(1.0 / b.v, -HUGE_VAL));
#else
  return CReal(a.v * std::nextafter(1.0 / b.v, HUGE_VAL));
#endif
#else
  return CReal(a.v / b.v);
#endif
}
static inline CReal& operator+=(CReal& a, CReal b) { a = a + b; return a; }
static inline CReal& operator-=(CReal& a, CReal b) { a = a - b; return a; }
static inline CReal& operator*=(CReal& a, CReal b) { a = a * b; return a; }
static inline CReal& operator/=(CReal& a, CReal b) { a = a / b; return a; }
#define ORC_CMP(op)                                                   \
  static inline bool operator op(CReal a, CReal b) {                  \
    ORC_TALLY(cmp);                                                   \
    return a.v op b.v;                                                \
  }
ORC_CMP(<) ORC_CMP(>) ORC_CMP(<=) ORC_CMP(>=) ORC_CMP(==) ORC_CMP(!=)
#undef ORC_CMP
#if defined(ORC_NUDGE)
/* the reciprocal build combined with transcendentals moved one ulp up */
static inline double cnudge(double v) { return std::nextafter(v, HUGE_VAL); }
#else
static inline double cnudge(double v) { return v; }
#endif
static inline CReal rexp(CReal x) { ORC_TALLY(transc); return CReal(cnudge(std::exp(x.v))); }
static inline CReal rlog(CReal x) { ORC_TALLY(transc); return CReal(cnudge(std::log(x.v))); }
static inline CReal rlog1p(CReal x) { ORC_TALLY(transc); return CReal(cnudge(std::log1p(x.v))); }
static inline CReal rpow(CReal x, CReal y) {
  ORC_TALLY(transc);
  return CReal(cnudge(std::pow(x.v, y.v)));
}
static inline CReal rsqrt(CReal x) { ORC_TALLY(sqrt_); return CReal(std::sqrt(x.v)); }
static inline double rval(CReal x) { return x.v; }

#endif

static inline real rabs(real x) { return x < real(0.0) ? -x : x; }
static inline real rmax(real a, real b) { return a < b ? b : a; }
static inline real rmin(real a, real b) { return b < a ? b : a; }

#endif
