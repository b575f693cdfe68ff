// FP operation count of the element arithmetic (sw_elem.h), for the
// algorithmic flops per tetrahedron the benchmark's ALU roofline uses:
// element_apply is instantiated on a number type that counts each addition,
// subtraction and multiplication (a fused multiply-add counts as two).
// Compiled with g++ by tests/test_flops.py against an empty stand-in for the
// HIP runtime header.
#include <cmath>
#include <cstdint>

using std::sqrt;

#define __host__
#define __device__
#define __forceinline__ inline

namespace {
int64_t g_ops = 0;
struct Cnt {
  double v;
  Cnt() : v(0) {}
  Cnt(double x) : v(x) {}
  Cnt(int x) : v(x) {}
  explicit operator double() const { return v; }
};
inline Cnt operator+(Cnt a, Cnt b) { ++g_ops; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g_ops; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g_ops; return Cnt(a.v * b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { ++g_ops; a.v += b.v; return a; }
inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }
}  // namespace

#include "sw_elem.h"

// flops of one element's stiffness and mass action (stiff, mass: which terms)
extern "C" int64_t element_flops(int stiff, int mass) {
  sw::Geo<Cnt> G;
  for (int j = 0; j < 4; ++j)
    for (int d = 0; d < 3; ++d) G.g[j][d] = Cnt(0.25 * (j + 1) + 0.5 * d);
  G.vol = Cnt(1.5);
  Cnt w[10][3];
  for (int k = 0; k < 10; ++k)
    for (int c = 0; c < 3; ++c) w[k][c] = Cnt(k + 0.25 * c);
  auto sink = [](int, Cnt, Cnt, Cnt) {};
  g_ops = 0;
  if (stiff && mass)
    sw::element_apply<Cnt, true, true, false>(G, Cnt(1.0), Cnt(2.0), Cnt(3.0), Cnt(4.0), w, sink);
  else if (stiff)
    sw::element_apply<Cnt, true, false, false>(G, Cnt(1.0), Cnt(2.0), Cnt(3.0), Cnt(4.0), w, sink);
  else if (mass)
    sw::element_apply<Cnt, false, true, false>(G, Cnt(1.0), Cnt(2.0), Cnt(3.0), Cnt(4.0), w, sink);
  return g_ops;
}
