// Operation count of the oracle's arithmetic (TEST INFRASTRUCTURE ONLY).
//
// Compiles euler_oracle.c unchanged as C++ with `double` replaced by a
// counting number type, so one call of orc_step tallies every floating-point
// operation the method performs on a given input.  The counts define the
// algorithmic work per cell-update used to place the GPU kernel on the
// arithmetic roofline; they never enter the HIP path.
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>

namespace fc {
struct Counts {
  long long add = 0, mul = 0, div = 0, sqrt = 0, cmp = 0;
};
static Counts g;

struct Num {
  double v;
  Num() = default;
  Num(double x) : v(x) {}
  Num(int x) : v(x) {}
  Num(long x) : v((double)x) {}
  Num(long long x) : v((double)x) {}
  explicit operator double() const { return v; }
};
inline Num operator+(Num a, Num b) { ++g.add; return Num(a.v + b.v); }
inline Num operator-(Num a, Num b) { ++g.add; return Num(a.v - b.v); }
inline Num operator*(Num a, Num b) { ++g.mul; return Num(a.v * b.v); }
inline Num operator/(Num a, Num b) { ++g.div; return Num(a.v / b.v); }
inline Num operator-(Num a) { return Num(-a.v); }
inline Num& operator+=(Num& a, Num b) { ++g.add; a.v += b.v; return a; }
inline Num& operator-=(Num& a, Num b) { ++g.add; a.v -= b.v; return a; }
inline Num& operator*=(Num& a, Num b) { ++g.mul; a.v *= b.v; return a; }
inline bool operator<(Num a, Num b) { ++g.cmp; return a.v < b.v; }
inline bool operator>(Num a, Num b) { ++g.cmp; return a.v > b.v; }
inline bool operator<=(Num a, Num b) { ++g.cmp; return a.v <= b.v; }
inline bool operator>=(Num a, Num b) { ++g.cmp; return a.v >= b.v; }
inline bool operator==(Num a, Num b) { ++g.cmp; return a.v == b.v; }
inline bool operator!=(Num a, Num b) { ++g.cmp; return a.v != b.v; }
inline Num sqrt(Num a) { ++g.sqrt; return Num(std::sqrt(a.v)); }
inline Num fabs(Num a) { ++g.cmp; return Num(std::fabs(a.v)); }
inline Num fmin(Num a, Num b) { ++g.cmp; return Num(std::fmin(a.v, b.v)); }
inline Num fmax(Num a, Num b) { ++g.cmp; return Num(std::fmax(a.v, b.v)); }
inline bool isfinite(Num a) { return std::isfinite(a.v); }
}  // namespace fc

using fc::fabs;
using fc::fmax;
using fc::fmin;
using fc::isfinite;
using fc::sqrt;

#define double fc::Num
#define isfinite(x) fc::isfinite(x)
// the analytic boundaries (sin, pow, the exact Riemann solver) are not part
// of the counted step
#define ORC_COUNTING 1
extern "C" {
#include "euler_oracle.c"
}
#undef double

extern "C" int orc_count_step(const orc_mesh* m, const fc::Num* U0, fc::Num dt, fc::Num* U2,
                              long long* counts) {
  fc::g = fc::Counts();
  int rc = orc_step(m, U0, dt, U2);
  counts[0] = fc::g.add;
  counts[1] = fc::g.mul;
  counts[2] = fc::g.div;
  counts[3] = fc::g.sqrt;
  counts[4] = fc::g.cmp;
  return rc;
}

extern "C" int orc_count_cfl(const orc_mesh* m, const fc::Num* U, fc::Num cfl, fc::Num* dt,
                             long long* counts) {
  fc::g = fc::Counts();
  int rc = orc_cfl_dt(m, U, cfl, dt);
  counts[0] = fc::g.add;
  counts[1] = fc::g.mul;
  counts[2] = fc::g.div;
  counts[3] = fc::g.sqrt;
  counts[4] = fc::g.cmp;
  return rc;
}
