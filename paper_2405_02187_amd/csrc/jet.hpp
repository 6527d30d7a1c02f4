// Complex-step numbers with a shared real part, for gfx950.
//
// A scalar is  x = x0 + sum_d x_d e_d + sum_{a<=b<Q} x_ab e_a e_b  with
// e_d^2 = 0 and e_a e_b kept only for a, b < Q.  This is the simplified
// complex arithmetic of Sec. 3 (eqs. "csfd_simplify_multiplication" and
// "csfd_simplify_division": products of two imaginary parts are dropped), with
// one imaginary unit per direction sharing a single real part, and the i1*i2
// part of the multicomplex expansion (eqs. "mc_taylor", "csfd_hessian") for the
// Hessian over the first Q directions.  x_d is h_d times the derivative along
// direction d; x_ab is h_a h_b times the mixed second derivative.
//
// The real part is evaluated with exactly the operations a real program would
// use (no FMA contraction on it; the library is compiled with
// -ffp-contract=off), so every decision taken on it matches a real run; the
// imaginary parts use explicit fma().
#pragma once
#include <hip/hip_runtime.h>

#define XJ __host__ __device__ __forceinline__

namespace xs {

template <typename T> XJ T tfma(T a, T b, T c) { return fma(a, b, c); }

template <typename T, int D, int Q>
struct Jet {
  static constexpr int P = Q * (Q + 1) / 2;
  static constexpr int N = 1 + D + P;
  T v[N];
  XJ T re() const { return v[0]; }
};

template <typename J> XJ J jzero() {
  J r;
#pragma unroll
  for (int c = 0; c < J::N; ++c) r.v[c] = 0;
  return r;
}
template <typename J, typename T> XJ J jconst(T c) {
  J r = jzero<J>();
  r.v[0] = c;
  return r;
}

template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator+(const Jet<T, D, Q>& x, const Jet<T, D, Q>& y) {
  Jet<T, D, Q> r;
#pragma unroll
  for (int c = 0; c < Jet<T, D, Q>::N; ++c) r.v[c] = x.v[c] + y.v[c];
  return r;
}
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator-(const Jet<T, D, Q>& x, const Jet<T, D, Q>& y) {
  Jet<T, D, Q> r;
#pragma unroll
  for (int c = 0; c < Jet<T, D, Q>::N; ++c) r.v[c] = x.v[c] - y.v[c];
  return r;
}
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator-(const Jet<T, D, Q>& x) {
  Jet<T, D, Q> r;
#pragma unroll
  for (int c = 0; c < Jet<T, D, Q>::N; ++c) r.v[c] = -x.v[c];
  return r;
}
// real scalar on either side
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator*(T s, const Jet<T, D, Q>& x) {
  Jet<T, D, Q> r;
#pragma unroll
  for (int c = 0; c < Jet<T, D, Q>::N; ++c) r.v[c] = s * x.v[c];
  return r;
}
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator*(const Jet<T, D, Q>& x, T s) { return s * x; }
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator+(const Jet<T, D, Q>& x, T s) { Jet<T, D, Q> r = x; r.v[0] = x.v[0] + s; return r; }
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator+(T s, const Jet<T, D, Q>& x) { Jet<T, D, Q> r = x; r.v[0] = s + x.v[0]; return r; }
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator-(const Jet<T, D, Q>& x, T s) { Jet<T, D, Q> r = x; r.v[0] = x.v[0] - s; return r; }
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator-(T s, const Jet<T, D, Q>& x) {
  Jet<T, D, Q> r = -x;
  r.v[0] = s - x.v[0];
  return r;
}

// product rule; second-order parts over pairs (a <= b < Q) in row-major order
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator*(const Jet<T, D, Q>& x, const Jet<T, D, Q>& y) {
  Jet<T, D, Q> r;
  const T x0 = x.v[0], y0 = y.v[0];
  r.v[0] = x0 * y0;
#pragma unroll
  for (int d = 1; d <= D; ++d) r.v[d] = tfma(x0, y.v[d], x.v[d] * y0);
  int p = 1 + D;
#pragma unroll
  for (int a = 0; a < Q; ++a)
#pragma unroll
    for (int b = a; b < Q; ++b, ++p) {
      T s = tfma(x0, y.v[p], x.v[p] * y0);
      s = tfma(x.v[1 + a], y.v[1 + b], s);
      r.v[p] = tfma(x.v[1 + b], y.v[1 + a], s);
    }
  return r;
}

// quotient q = x / y: q0 by an IEEE division; parts from x = q y
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator/(const Jet<T, D, Q>& x, const Jet<T, D, Q>& y) {
  Jet<T, D, Q> q;
  const T y0 = y.v[0];
  q.v[0] = x.v[0] / y0;
  const T inv = T(1) / y0;
  const T q0 = q.v[0];
#pragma unroll
  for (int d = 1; d <= D; ++d) q.v[d] = tfma(-q0, y.v[d], x.v[d]) * inv;
  int p = 1 + D;
#pragma unroll
  for (int a = 0; a < Q; ++a)
#pragma unroll
    for (int b = a; b < Q; ++b, ++p) {
      T s = tfma(-q0, y.v[p], x.v[p]);
      s = tfma(-q.v[1 + a], y.v[1 + b], s);
      s = tfma(-q.v[1 + b], y.v[1 + a], s);
      q.v[p] = s * inv;
    }
  return q;
}
template <typename T, int D, int Q>
XJ Jet<T, D, Q> operator/(const Jet<T, D, Q>& x, T s) {
  Jet<T, D, Q> r;
  r.v[0] = x.v[0] / s;
  const T inv = T(1) / s;
#pragma unroll
  for (int c = 1; c < Jet<T, D, Q>::N; ++c) r.v[c] = x.v[c] * inv;
  return r;
}

// f(x) given f(x0), f'(x0), f''(x0)
template <typename T, int D, int Q>
XJ Jet<T, D, Q> chain(const Jet<T, D, Q>& x, T f0, T f1, T f2) {
  Jet<T, D, Q> r;
  r.v[0] = f0;
#pragma unroll
  for (int d = 1; d <= D; ++d) r.v[d] = f1 * x.v[d];
  int p = 1 + D;
#pragma unroll
  for (int a = 0; a < Q; ++a)
#pragma unroll
    for (int b = a; b < Q; ++b, ++p) r.v[p] = tfma(f2 * x.v[1 + a], x.v[1 + b], f1 * x.v[p]);
  return r;
}
template <typename T, int D, int Q> XJ Jet<T, D, Q> jsqrt(const Jet<T, D, Q>& x) {
  T s = sqrt(x.v[0]);
  T f1 = T(0.5) / s;
  return chain(x, s, f1, -f1 / (T(2) * x.v[0]));
}
template <typename T, int D, int Q> XJ Jet<T, D, Q> jexp(const Jet<T, D, Q>& x) {
  T e = exp(x.v[0]);
  return chain(x, e, e, e);
}
template <typename T, int D, int Q> XJ Jet<T, D, Q> jsin(const Jet<T, D, Q>& x) {
  T s = sin(x.v[0]), c = cos(x.v[0]);
  return chain(x, s, c, -s);
}
template <typename T, int D, int Q> XJ Jet<T, D, Q> jcos(const Jet<T, D, Q>& x) {
  T s = sin(x.v[0]), c = cos(x.v[0]);
  return chain(x, c, -s, -c);
}

// precision conversion (FP64 master pose -> kernel precision)
template <typename T, typename U, int D, int Q> XJ Jet<T, D, Q> jcast(const Jet<U, D, Q>& x) {
  Jet<T, D, Q> r;
#pragma unroll
  for (int c = 0; c < Jet<T, D, Q>::N; ++c) r.v[c] = T(x.v[c]);
  return r;
}

// ---- 3-vectors of jets -------------------------------------------------------
template <typename J> struct V3 { J x, y, z; };
template <typename J> XJ V3<J> vadd(const V3<J>& a, const V3<J>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename J> XJ V3<J> vsub(const V3<J>& a, const V3<J>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename J> XJ V3<J> vscale(const J& s, const V3<J>& a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename J> XJ J vdot(const V3<J>& a, const V3<J>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename J> XJ V3<J> vcross(const V3<J>& a, const V3<J>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// ---- SoA loads / stores: component c of element i at base[c * stride + i] ---
template <typename J, typename T> XJ J jload(const T* base, size_t stride, size_t i) {
  J r;
#pragma unroll
  for (int c = 0; c < J::N; ++c) r.v[c] = base[c * stride + i];
  return r;
}
template <typename J, typename T> XJ void jstore(T* base, size_t stride, size_t i, const J& x) {
#pragma unroll
  for (int c = 0; c < J::N; ++c) base[c * stride + i] = x.v[c];
}
// 3-vector map: component planes of x, then y, then z
template <typename J, typename T> XJ V3<J> vload(const T* base, size_t stride, size_t i) {
  return {jload<J>(base, stride, i), jload<J>(base + J::N * stride, stride, i),
          jload<J>(base + 2 * J::N * stride, stride, i)};
}
// ---- loads that share one memory round trip ----------------------------------
// pin() hands a loaded value to an empty asm statement that reads its VGPRs:
// the load must then be issued before that point, so a later branch that does
// not need the value cannot pull the load below itself (the compiler sinks
// loads into the branch that uses them, one round trip per branch).  Loads
// written side by side and pinned together wait once.
__device__ __forceinline__ void pin(float& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(uint32_t& x) { asm volatile("" : "+v"(x)); }
template <typename T, int D, int Q> __device__ __forceinline__ void pin(Jet<T, D, Q>& x) {
#pragma unroll
  for (int c = 0; c < Jet<T, D, Q>::N; ++c) pin(x.v[c]);
}
template <typename J> __device__ __forceinline__ void pin(V3<J>& a) {
  pin(a.x);
  pin(a.y);
  pin(a.z);
}

template <typename J, typename T> XJ void vstore(T* base, size_t stride, size_t i, const V3<J>& v) {
  jstore(base, stride, i, v.x);
  jstore(base + J::N * stride, stride, i, v.y);
  jstore(base + 2 * J::N * stride, stride, i, v.z);
}

}  // namespace xs
