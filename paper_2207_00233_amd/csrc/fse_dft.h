// fse_dft.h -- small complex DFTs in double held in one thread's registers,
// shared by the FP64 transform pass of the 2-D path and the 3-D kernel.
#pragma once
#include <hip/hip_runtime.h>

namespace fse {
namespace dft {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
// v e^{-j theta} with t = (cos theta, sin theta)
__device__ __forceinline__ double2 cmul_conj(double2 v, double2 t) {
  return make_double2(fma(v.x, t.x, v.y * t.y), fma(v.y, t.x, -v.x * t.y));
}
__device__ __forceinline__ double2 mul_mj(double2 v) { return make_double2(v.y, -v.x); }  // -j v

// y[k] = sum_n x[n] e^{-j 2 pi n k / 4}, in place
__device__ __forceinline__ void dft4(double2& x0, double2& x1, double2& x2, double2& x3) {
  const double2 a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = mul_mj(csub(x1, x3));
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, d);
  x3 = csub(b, d);
}

// y[k] = sum_n x[n] e^{-j 2 pi n k / 8}, in place: 4-point DFTs of the even
// and odd samples joined with the factors e^{-j 2 pi k / 8}
__device__ __forceinline__ void dft8(double2 (&v)[8]) {
  constexpr double c = 0.70710678118654752440;  // 1 / sqrt(2)
  double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  o1 = make_double2(c * (o1.x + o1.y), c * (o1.y - o1.x));   // e^{-j pi / 4}
  o2 = mul_mj(o2);                                           // e^{-j pi / 2}
  o3 = make_double2(c * (o3.y - o3.x), -c * (o3.x + o3.y));  // e^{-j 3 pi / 4}
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

}  // namespace dft
}  // namespace fse
