/*
 * orc_real.h -- scalar type of the oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The plain build uses `real` = double.  The counting build (-DORC_COUNT)
 * replaces it by a class that performs the same binary64 arithmetic and
 * counts each operation, so that the algorithmic operation count per
 * cell-update comes from the very code that defines the method.
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
static inline real rexp(real x) { return std::exp(x); }
static inline real rlog(real x) { return std::log(x); }
static inline real rlog1p(real x) { return std::log1p(x); }
static inline real rpow(real x, real y) { return std::pow(x, y); }
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
