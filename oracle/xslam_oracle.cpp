// CPU oracle for the CSFD dense-SLAM frame step (X-SLAM, Sec. 3 and Sec. 4.1).
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or call
// this code: only the test-suite, the smoke check and the benchmark's CPU
// baseline leg use it.  It shares no code, header, table or helper with the GPU
// library.
//
// What it is: the KinectFusion-style frame step of Sec. 4.1 written as plain
// nested loops over one scalar type S, instantiated for
//   S = double                    (real run; central finite differences),
//   S = std::complex<double>      (CSFD first derivative, Sec. 3 eq. "csfd",
//                                  with FULL complex arithmetic and the standard
//                                  library's complex elementary functions; it
//                                  deliberately does not use the simplified
//                                  products of eqs. "csfd_simplify_*"),
//   S = Bicomplex                 (second derivatives, Sec. 3 eqs.
//                                  "multi_complex", "mc_taylor", "csfd_hessian").
// Every branch, floor and validity test is decided on the real part.  The
// readings of the passages the paper leaves open are listed next to each step.
//
// Parity pins: see tests/test_oracle_*.py (closed forms, FD sweeps, Hessian
// symmetry, known-pose ICP recovery).

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

typedef std::complex<double> cd;

// ---------------------------------------------------------------------------
// Bicomplex numbers z1 + z2 i2 with z1, z2 in C(i1)   (Sec. 3, eq. multi_complex)
// ---------------------------------------------------------------------------
struct Bicomplex {
  cd a, b;  // a + b*i2
  Bicomplex() : a(0.0), b(0.0) {}
  Bicomplex(double x) : a(x), b(0.0) {}
  Bicomplex(cd x, cd y) : a(x), b(y) {}
};
inline Bicomplex operator+(const Bicomplex& x, const Bicomplex& y) { return {x.a + y.a, x.b + y.b}; }
inline Bicomplex operator-(const Bicomplex& x, const Bicomplex& y) { return {x.a - y.a, x.b - y.b}; }
inline Bicomplex operator-(const Bicomplex& x) { return {-x.a, -x.b}; }
inline Bicomplex operator*(const Bicomplex& x, const Bicomplex& y) {
  return {x.a * y.a - x.b * y.b, x.a * y.b + x.b * y.a};  // i2^2 = -1, exact product
}
inline Bicomplex operator/(const Bicomplex& x, const Bicomplex& y) {
  // The exact quotient q = x / y of q y = x:
  //   q.b = (x.b y.a - x.a y.b) / (y.a^2 + y.b^2),   q.a = (x.a + q.b y.b) / y.a.
  // Written this way (not as x times 1/y) the real part of q is the real
  // quotient re(x)/re(y) of a real run, so that every decision taken on real
  // parts is the real run's.
  const cd qb = (x.b * y.a - x.a * y.b) / (y.a * y.a + y.b * y.b);
  const cd qa = (x.a + qb * y.b) / y.a;
  return {qa, qb};
}
inline Bicomplex& operator+=(Bicomplex& x, const Bicomplex& y) { x = x + y; return x; }
inline Bicomplex& operator-=(Bicomplex& x, const Bicomplex& y) { x = x - y; return x; }
inline Bicomplex& operator*=(Bicomplex& x, const Bicomplex& y) { x = x * y; return x; }
// Elementary functions by Taylor expansion in the i2 part:
//   f(a + b i2) = f(a) - f''(a) b^2 / 2 + i2 f'(a) b      (truncation O(b^3)).
// f, f', f'' are complex (C(i1)) standard-library evaluations.  The idempotent
// split f(a -+ i1 b) is not used: its i1*i2 part is a difference of nearly
// equal numbers and vanishes at tiny steps.
inline Bicomplex taylor2(const cd& f, const cd& f1, const cd& f2, const Bicomplex& z) {
  return {f - f2 * z.b * z.b * 0.5, f1 * z.b};
}
inline Bicomplex sqrt(const Bicomplex& z) {
  cd s = std::sqrt(z.a);
  return taylor2(s, 0.5 / s, -0.25 / (s * z.a), z);
}
inline Bicomplex exp(const Bicomplex& z) { cd e = std::exp(z.a); return taylor2(e, e, e, z); }
inline Bicomplex sin(const Bicomplex& z) {
  cd s = std::sin(z.a), c = std::cos(z.a);
  return taylor2(s, c, -s, z);
}
inline Bicomplex cos(const Bicomplex& z) {
  cd s = std::sin(z.a), c = std::cos(z.a);
  return taylor2(c, -s, -c, z);
}

// real part used for every decision
inline double re(double x) { return x; }
inline double re(const cd& x) { return x.real(); }
inline double re(const Bicomplex& x) { return x.a.real(); }

inline double sqrt(double x) { return std::sqrt(x); }
inline double exp(double x) { return std::exp(x); }
inline double sin(double x) { return std::sin(x); }
inline double cos(double x) { return std::cos(x); }
inline cd sqrt(const cd& x) { return std::sqrt(x); }
inline cd exp(const cd& x) { return std::exp(x); }
inline cd sin(const cd& x) { return std::sin(x); }
inline cd cos(const cd& x) { return std::cos(x); }

// number of doubles per scalar in the C interface: (re), (re, im), (re, i1, i2, i1i2)
template <class S> struct NC;
template <> struct NC<double> { static constexpr int n = 1; };
template <> struct NC<cd> { static constexpr int n = 2; };
template <> struct NC<Bicomplex> { static constexpr int n = 4; };

inline void put(double* p, double x) { p[0] = x; }
inline void put(double* p, const cd& x) { p[0] = x.real(); p[1] = x.imag(); }
inline void put(double* p, const Bicomplex& x) { p[0] = x.a.real(); p[1] = x.a.imag(); p[2] = x.b.real(); p[3] = x.b.imag(); }
template <class S> S get(const double* p);
template <> inline double get<double>(const double* p) { return p[0]; }
template <> inline cd get<cd>(const double* p) { return cd(p[0], p[1]); }
template <> inline Bicomplex get<Bicomplex>(const double* p) { return Bicomplex(cd(p[0], p[1]), cd(p[2], p[3])); }

// perturbation of a real value: + h on i1 (complex: i) and/or + h on i2
template <class S> S seeded(double x, double d1, double d2);
template <> inline double seeded<double>(double x, double, double) { return x; }
template <> inline cd seeded<cd>(double x, double d1, double) { return cd(x, d1); }
template <> inline Bicomplex seeded<Bicomplex>(double x, double d1, double d2) { return Bicomplex(cd(x, d1), cd(d2, 0.0)); }

// ---------------------------------------------------------------------------
// small vector / matrix helpers (bilinear, no conjugation anywhere)
// ---------------------------------------------------------------------------
template <class S> struct V3 {
  S x, y, z;
  V3() : x(0.0), y(0.0), z(0.0) {}
  V3(S a, S b, S c) : x(a), y(b), z(c) {}
};
template <class S> V3<S> operator+(const V3<S>& a, const V3<S>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class S> V3<S> operator-(const V3<S>& a, const V3<S>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S> V3<S> operator*(const S& s, const V3<S>& a) { return {s * a.x, s * a.y, s * a.z}; }
template <class S> S dot(const V3<S>& a, const V3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// 4x4 rigid transform, camera-to-world, row-major
template <class S> struct M4 {
  S m[16];
  M4() { for (int i = 0; i < 16; ++i) m[i] = S(0.0); m[0] = m[5] = m[10] = m[15] = S(1.0); }
  S& operator()(int r, int c) { return m[r * 4 + c]; }
  const S& operator()(int r, int c) const { return m[r * 4 + c]; }
};
template <class S> M4<S> mul(const M4<S>& A, const M4<S>& B) {
  M4<S> C;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      S s(0.0);
      for (int k = 0; k < 4; ++k) s = s + A(r, k) * B(k, c);
      C(r, c) = s;
    }
  return C;
}
template <class S> V3<S> apply(const M4<S>& T, const V3<S>& p) {  // R p + t
  return {T(0, 0) * p.x + T(0, 1) * p.y + T(0, 2) * p.z + T(0, 3),
          T(1, 0) * p.x + T(1, 1) * p.y + T(1, 2) * p.z + T(1, 3),
          T(2, 0) * p.x + T(2, 1) * p.y + T(2, 2) * p.z + T(2, 3)};
}
template <class S> V3<S> rotate(const M4<S>& T, const V3<S>& p) {  // R p
  return {T(0, 0) * p.x + T(0, 1) * p.y + T(0, 2) * p.z,
          T(1, 0) * p.x + T(1, 1) * p.y + T(1, 2) * p.z,
          T(2, 0) * p.x + T(2, 1) * p.y + T(2, 2) * p.z};
}
template <class S> V3<S> apply_inv(const M4<S>& T, const V3<S>& p) {  // R^T (p - t), transpose not conjugate
  V3<S> d(p.x - T(0, 3), p.y - T(1, 3), p.z - T(2, 3));
  return {T(0, 0) * d.x + T(1, 0) * d.y + T(2, 0) * d.z,
          T(0, 1) * d.x + T(1, 1) * d.y + T(2, 1) * d.z,
          T(0, 2) * d.x + T(1, 2) * d.y + T(2, 2) * d.z};
}
template <class S> M4<S> inverse(const M4<S>& T) {
  M4<S> I;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) I(r, c) = T(c, r);
  for (int r = 0; r < 3; ++r) I(r, 3) = -(I(r, 0) * T(0, 3) + I(r, 1) * T(1, 3) + I(r, 2) * T(2, 3));
  return I;
}

// ---------------------------------------------------------------------------
// SE(3) exponential (Sec. 4.1 eqs. "lie", "rotvector", "rotation_jacobi")
//   theta^2 = phi . phi (bilinear); R = I + A[phi]x + B[phi]x^2;
//   V = I + B[phi]x + C[phi]x^2 (the rotation Jacobian of eq. rotation_jacobi,
//   using a a^T = I + [a]x^2 with a plain transpose); t = V rho.
//   A = sin(th)/th, B = (1-cos th)/th^2, C = (th - sin th)/th^3, as even series
//   in theta^2 when re(theta^2) < 1e-2 (the axis a = phi/theta is undefined at
//   phi = 0 and the arccos form of theta is circular).
// ---------------------------------------------------------------------------
template <class S> M4<S> se3_exp(const S xi[6]) {
  V3<S> ph(xi[0], xi[1], xi[2]), rh(xi[3], xi[4], xi[5]);
  S t2 = dot(ph, ph);
  S A, B, C;
  if (re(t2) < 1e-2) {
    S t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4;
    A = S(1.0) - t2 / S(6.0) + t4 / S(120.0) - t6 / S(5040.0) + t8 / S(362880.0);
    B = S(0.5) - t2 / S(24.0) + t4 / S(720.0) - t6 / S(40320.0) + t8 / S(3628800.0);
    C = S(1.0 / 6.0) - t2 / S(120.0) + t4 / S(5040.0) - t6 / S(362880.0) + t8 / S(39916800.0);
  } else {
    S th = sqrt(t2);
    S s = sin(th), c = cos(th);
    A = s / th;
    B = (S(1.0) - c) / t2;
    C = (th - s) / (t2 * th);
  }
  // [phi]x and [phi]x^2
  S K[3][3] = {{S(0.0), -ph.z, ph.y}, {ph.z, S(0.0), -ph.x}, {-ph.y, ph.x, S(0.0)}};
  S K2[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      S s(0.0);
      for (int k = 0; k < 3; ++k) s = s + K[r][k] * K[k][c];
      K2[r][c] = s;
    }
  M4<S> T;
  S Vm[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      S I = S(r == c ? 1.0 : 0.0);
      T(r, c) = I + A * K[r][c] + B * K2[r][c];
      Vm[r][c] = I + B * K[r][c] + C * K2[r][c];
    }
  S rr[3] = {rh.x, rh.y, rh.z};
  for (int r = 0; r < 3; ++r) T(r, 3) = Vm[r][0] * rr[0] + Vm[r][1] * rr[1] + Vm[r][2] * rr[2];
  return T;
}

// Small-angle transform of eq. icp_approx (the original KinectFusion
// linearisation): cos of each angle taken as 1 and sin as the angle, i.e.
// rotation I + [phi]x and translation rho.
template <class S> M4<S> small_angle(const S xi[6]) {
  M4<S> T;
  T(0, 1) = -xi[2]; T(0, 2) = xi[1];
  T(1, 0) = xi[2];  T(1, 2) = -xi[0];
  T(2, 0) = -xi[1]; T(2, 1) = xi[0];
  for (int r = 0; r < 3; ++r) T(r, 3) = xi[3 + r];
  return T;
}

// ---------------------------------------------------------------------------
// configuration and seeding
// ---------------------------------------------------------------------------
enum Param {
  P_PHI_X = 0, P_PHI_Y, P_PHI_Z, P_RHO_X, P_RHO_Y, P_RHO_Z,
  P_TRUNC = 6, P_WCAP = 7, P_DGATE = 8, P_AGATE = 9,
  P_ICPW0 = 10, P_ICPW1 = 11, P_ICPW2 = 12,
  P_FX = 13, P_FY = 14, P_CX = 15, P_CY = 16, P_DEPTH = 17
};

}  // namespace orc

extern "C" {
struct OrcConfig {
  int32_t width, height;
  double fx, fy, cx, cy;
  int32_t dim[3];
  double voxel, trunc, wcap;
  int32_t iters[3];          // per level, level 0 = finest; levels run coarse to fine
  double dgate, agate_deg;   // ICP gates
  double level_w[3];         // per-level step relaxation
  double disc_delta;         // discontinuity threshold for bilinear lookups (m)
  int32_t bilateral_radius;
  double sigma_px, sigma_m;  // bilateral spatial (pixels) and range (m) sigmas
  double near_m;             // raycast near plane
  int32_t init;              // 0 previous pose, 1 constant velocity
  int32_t update;            // 0 exact exponential, 1 small-angle matrix (eq. icp_approx) + polar steps
  int32_t solver;            // 0 Gauss-Newton; Newton with the complex-step Hessian (real runs only):
                             // 1 correspondences held fixed per pass, 2 through the association
  // surfel front end (X-PointFusion)
  double pf_d_depth;         // candidate filter: depth difference along the viewing ray (m)
  double pf_d_norm_deg;      // candidate filter: normal deviation (degrees)
  double pf_d_dist;          // candidate filter: distance to the measured point (m)
  double pf_sigma;           // Gaussian kernel of the one-to-many weights (m)
  double pf_c_stable;        // confidence a surfel needs to enter the predicted model maps
  int32_t pf_capacity;       // maximum number of surfels
};
struct OrcSeed {
  int32_t kind;  // 0 real, 1 complex (direction pa), 2 bicomplex (pa on i1, pb on i2)
  int32_t pa, pb;
  double h;
};
}

namespace orc {

struct Ctx {
  OrcConfig c;
  OrcSeed s;
  double d1(int p) const { return (s.kind >= 1 && s.pa == p) ? s.h : 0.0; }
  double d2(int p) const { return (s.kind == 2 && s.pb == p) ? s.h : 0.0; }
  template <class S> S par(double v, int p) const { return seeded<S>(v, d1(p), d2(p)); }
};

template <class S> struct Params {
  S fx, fy, cx, cy, mu, wcap, dgate, agate, w[3];
};
template <class S> Params<S> make_params(const Ctx& X) {
  Params<S> P;
  P.fx = X.par<S>(X.c.fx, P_FX); P.fy = X.par<S>(X.c.fy, P_FY);
  P.cx = X.par<S>(X.c.cx, P_CX); P.cy = X.par<S>(X.c.cy, P_CY);
  P.mu = X.par<S>(X.c.trunc, P_TRUNC); P.wcap = X.par<S>(X.c.wcap, P_WCAP);
  P.dgate = X.par<S>(X.c.dgate, P_DGATE); P.agate = X.par<S>(X.c.agate_deg, P_AGATE);
  for (int l = 0; l < 3; ++l) P.w[l] = X.par<S>(X.c.level_w[l], P_ICPW0 + l);
  return P;
}

// intrinsics of pyramid level l: K / 2^l (pixel centres at integers)
template <class S> struct Intr { S fx, fy, cx, cy; int W, H; };
template <class S> Intr<S> level_intr(const Params<S>& P, const OrcConfig& c, int l) {
  double s = 1.0 / double(1 << l);
  return {P.fx * S(s), P.fy * S(s), P.cx * S(s), P.cy * S(s), c.width >> l, c.height >> l};
}

inline bool valid_depth(double d) { return d > 0.0 && std::isfinite(d); }

// ---------------------------------------------------------------------------
// A1. depth promotion (eq. csfd_depth), bilateral filter, pyramid
// ---------------------------------------------------------------------------
// D*(u) = D(u) + i h Ddot(u): the caller supplies the tangent plane Ddot.
template <class S> std::vector<S> promote_depth(const Ctx& X, const double* D, const double* Ddot) {
  int n = X.c.width * X.c.height;
  std::vector<S> out(n, S(0.0));
  for (int i = 0; i < n; ++i) {
    if (!valid_depth(D[i])) continue;
    double t = Ddot ? Ddot[i] : 0.0;
    out[i] = seeded<S>(D[i], X.d1(P_DEPTH) * t, X.d2(P_DEPTH) * t);
  }
  return out;
}

// Bilateral filter of the raw depth (Sec. 4.1 "Surface measurement"): normalised
// sum over valid pixels of a (2r+1)^2 window, weights
// exp(-|u-u'|^2/(2 sigma_px^2) - (D(u)-D(u'))^2/(2 sigma_m^2)), complex through D.
template <class S> std::vector<S> bilateral(const Ctx& X, const std::vector<S>& D) {
  int W = X.c.width, H = X.c.height, r = X.c.bilateral_radius;
  if (r <= 0) return D;
  double is = 1.0 / (2.0 * X.c.sigma_px * X.c.sigma_px), ir = 1.0 / (2.0 * X.c.sigma_m * X.c.sigma_m);
  std::vector<S> out(W * H, S(0.0));
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const S& c = D[y * W + x];
      if (!(re(c) > 0.0)) continue;
      S num(0.0), den(0.0);
      for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
          int xx = x + dx, yy = y + dy;
          if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
          const S& d = D[yy * W + xx];
          if (!(re(d) > 0.0)) continue;
          S dd = c - d;
          S w = exp(-(S(double(dx * dx + dy * dy) * is) + dd * dd * S(ir)));
          num = num + w * d;
          den = den + w;
        }
      out[y * W + x] = num / den;
    }
  return out;
}

// Coarser level (Sec. 4.1: "Gaussian smoothing", the perturbation smoothed too):
// 5x5 binomial (1,4,6,4,1)^2 centred on (2x,2y), valid taps within 3 sigma_m of
// the centre, renormalised; real weights.
template <class S> std::vector<S> pyrdown(const Ctx& X, const std::vector<S>& D, int W, int H) {
  static const int g[5] = {1, 4, 6, 4, 1};
  int W2 = W / 2, H2 = H / 2;
  std::vector<S> out(W2 * H2, S(0.0));
  double gate = 3.0 * X.c.sigma_m;
  for (int y = 0; y < H2; ++y)
    for (int x = 0; x < W2; ++x) {
      const S& c = D[(2 * y) * W + 2 * x];
      if (!(re(c) > 0.0)) continue;
      S num(0.0);
      double den = 0.0;
      for (int j = -2; j <= 2; ++j)
        for (int i = -2; i <= 2; ++i) {
          int xx = 2 * x + i, yy = 2 * y + j;
          if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
          const S& d = D[yy * W + xx];
          if (!(re(d) > 0.0)) continue;
          if (std::fabs(re(d) - re(c)) > gate) continue;
          double w = double(g[i + 2] * g[j + 2]);
          num = num + S(w) * d;
          den += w;
        }
      out[y * W2 + x] = num / S(den);
    }
  return out;
}

// ---------------------------------------------------------------------------
// A2. vertex and normal maps (eqs. vertex, normal)
//   V(u) = D(u) K^-1 (u,1);  N = normalize((V(u_y+) - V(u)) x (V(u_x+) - V(u)))
//   (operands ordered so that the normal faces the camera, like grad F).
// ---------------------------------------------------------------------------
template <class S> struct Maps {
  int W = 0, H = 0;
  std::vector<V3<S>> V, N;
  std::vector<uint8_t> valid;   // vertex validity (V) and normal validity (N) combined for ICP use
  std::vector<uint8_t> vvalid;
  std::vector<double> Z;        // model maps only: camera depth of the hit (real)
};

template <class S> Maps<S> vertex_normal(const std::vector<S>& D, const Intr<S>& K) {
  Maps<S> M;
  M.W = K.W; M.H = K.H;
  int n = K.W * K.H;
  M.V.assign(n, V3<S>()); M.N.assign(n, V3<S>()); M.valid.assign(n, 0); M.vvalid.assign(n, 0);
  for (int y = 0; y < K.H; ++y)
    for (int x = 0; x < K.W; ++x) {
      const S& d = D[y * K.W + x];
      if (!(re(d) > 0.0)) continue;
      V3<S> ray((S(double(x)) - K.cx) / K.fx, (S(double(y)) - K.cy) / K.fy, S(1.0));
      M.V[y * K.W + x] = d * ray;
      M.vvalid[y * K.W + x] = 1;
    }
  for (int y = 0; y + 1 < K.H; ++y)
    for (int x = 0; x + 1 < K.W; ++x) {
      int i = y * K.W + x;
      if (!M.vvalid[i] || !M.vvalid[i + 1] || !M.vvalid[i + K.W]) continue;
      V3<S> a = M.V[i + 1] - M.V[i], b = M.V[i + K.W] - M.V[i];
      V3<S> c = cross(b, a);
      S cc = dot(c, c);
      if (!(re(cc) > 0.0)) continue;
      S inv = S(1.0) / sqrt(cc);
      M.N[i] = inv * c;
      M.valid[i] = 1;
    }
  return M;
}

// ---------------------------------------------------------------------------
// A3/A4. projective association + point-to-plane residual + normal equations
// (eq. icp and the passage after eq. icp_approx).  One pass over the current
// level in row-major order.  Returns A (21, upper triangle row-major), b (6).
// ---------------------------------------------------------------------------
template <class S> struct Normal {
  S A[21], b[6];
  int64_t cnt = 0;
  double r2 = 0.0;
  Normal() { for (auto& a : A) a = S(0.0); for (auto& x : b) x = S(0.0); }
};

// bilinear lookup of a 3-vector model map at u (complex fractions) with the
// discontinuity rule of Sec. 4.1 ("derivative w.r.t. pixel coordinate"): when
// sum_taps |z(tap) - z(nearest)| >= delta the nearest tap is used unperturbed.
// Returns false if a tap is outside or invalid.
template <class S> struct Lookup { V3<S> q, m; };

// The tap row/column is floor(u + 1e-3): at the first iteration of a level
// (T_j = T_{k-1}) every pixel re-projects onto its own integer coordinate up to
// rounding, and a plain floor would pick the left or right cell by rounding
// noise; the bias moves that tie a thousandth of a pixel away from the integers.
const double kTapBias = 1e-3;

template <class S>
bool model_lookup(const Maps<S>& M, const S& ux, const S& uy, double delta, Lookup<S>& out, bool hold = false) {
  double rx = re(ux), ry = re(uy);
  double fx0 = std::floor(rx + kTapBias), fy0 = std::floor(ry + kTapBias);
  if (!(fx0 >= 0.0 && fy0 >= 0.0 && fx0 <= double(M.W - 2) && fy0 <= double(M.H - 2))) return false;
  int i0 = int(fx0), j0 = int(fy0);
  int t[4] = {j0 * M.W + i0, j0 * M.W + i0 + 1, (j0 + 1) * M.W + i0, (j0 + 1) * M.W + i0 + 1};
  for (int k = 0; k < 4; ++k)
    if (!M.valid[t[k]]) return false;
  int in = int(std::floor(rx + 0.5)), jn = int(std::floor(ry + 0.5));
  int tn = jn * M.W + in;
  double disc = 0.0;
  for (int k = 0; k < 4; ++k) disc += std::fabs(M.Z[t[k]] - M.Z[tn]);
  if (disc >= delta) {
    out.q = M.V[tn];
    out.m = M.N[tn];
    return true;
  }
  // hold: the fractional position taken from the real parts, so the
  // looked-up point and normal do not move with the pose (the Newton step of
  // one ICP pass with its correspondences held fixed)
  S a = hold ? S(rx - double(i0)) : ux - S(double(i0));
  S b = hold ? S(ry - double(j0)) : uy - S(double(j0));
  S a1 = S(1.0) - a, b1 = S(1.0) - b;
  out.q = b1 * (a1 * M.V[t[0]] + a * M.V[t[1]]) + b * (a1 * M.V[t[2]] + a * M.V[t[3]]);
  V3<S> m = b1 * (a1 * M.N[t[0]] + a * M.N[t[1]]) + b * (a1 * M.N[t[2]] + a * M.N[t[3]]);
  out.m = (S(1.0) / sqrt(dot(m, m))) * m;
  return true;
}

// Point-to-plane residual of current pixel i at pose T (eq. icp): false if the
// pixel has no correspondence (invalid, behind, outside, invalid taps, gates).
// J = [p x m; m] is the Jacobian of the residual for the left increment with
// the correspondence held fixed (the Gauss-Newton linearisation).
template <class S>
bool icp_residual(const Ctx& X, const Params<S>& P, const Maps<S>& cur, const Maps<S>& model, const Intr<S>& K,
                  const M4<S>& Tprev, const M4<S>& T, int i, S& r, S J[6], bool hold = false) {
  double dg = re(P.dgate);
  double dg2 = dg * dg;
  double cosa = std::cos(re(P.agate) * M_PI / 180.0);
  if (!cur.valid[i]) return false;
  V3<S> p = apply(T, cur.V[i]);
  V3<S> n = rotate(T, cur.N[i]);
  V3<S> xc = apply_inv(Tprev, p);
  if (!(re(xc.z) > 0.0)) return false;
  S ux = K.fx * xc.x / xc.z + K.cx;
  S uy = K.fy * xc.y / xc.z + K.cy;
  Lookup<S> L;
  if (!model_lookup(model, ux, uy, X.c.disc_delta, L, hold)) return false;
  V3<S> d = p - L.q;
  if (!(re(dot(d, d)) <= dg2)) return false;
  if (!(re(dot(n, L.m)) >= cosa)) return false;
  r = dot(d, L.m);
  V3<S> pm = cross(p, L.m);
  J[0] = pm.x; J[1] = pm.y; J[2] = pm.z; J[3] = L.m.x; J[4] = L.m.y; J[5] = L.m.z;
  return true;
}

template <class S>
Normal<S> icp_reduce(const Ctx& X, const Params<S>& P, const Maps<S>& cur, const Maps<S>& model,
                     const Intr<S>& K, const M4<S>& Tprev, const M4<S>& T) {
  Normal<S> E;
  for (int y = 0; y < cur.H; ++y)
    for (int x = 0; x < cur.W; ++x) {
      int i = y * cur.W + x;
      S r, J[6];
      if (!icp_residual(X, P, cur, model, K, Tprev, T, i, r, J)) continue;
      int k = 0;
      for (int a = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b) E.A[k++] += J[a] * J[b];
      for (int a = 0; a < 6; ++a) E.b[a] += J[a] * r;
      E.cnt += 1;
      E.r2 += re(r) * re(r);
    }
  return E;
}

// A5. solve A delta = -b by Gaussian elimination without pivoting and without
// conjugation (the normal matrix is symmetric positive definite in its real
// part).  Lost when a pivot's real part <= 1e-12 * max real diagonal.
template <class S> bool solve6(const S Au[21], const S b[6], S x[6]) {
  S A[6][7];
  int k = 0;
  for (int a = 0; a < 6; ++a)
    for (int c = a; c < 6; ++c) { A[a][c] = Au[k]; A[c][a] = Au[k]; ++k; }
  for (int a = 0; a < 6; ++a) A[a][6] = -b[a];
  double dmax = 0.0;
  for (int a = 0; a < 6; ++a) dmax = std::max(dmax, re(A[a][a]));
  for (int c = 0; c < 6; ++c) {
    if (!(re(A[c][c]) > 1e-12 * dmax)) return false;
    for (int r = c + 1; r < 6; ++r) {
      S f = A[r][c] / A[c][c];
      for (int j = c; j < 7; ++j) A[r][j] = A[r][j] - f * A[c][j];
    }
  }
  for (int r = 5; r >= 0; --r) {
    S s = A[r][6];
    for (int j = r + 1; j < 6; ++j) s = s - A[r][j] * x[j];
    x[r] = s / A[r][r];
  }
  return true;
}

// ---------------------------------------------------------------------------
// Newton ICP (Sec. 4.1: a second-order ICP with Newton's method at each ICP
// step, its Hessian by the multicomplex step of eq. csfd_hessian, and no
// small-angle approximation).  The objective of one pass is
// E(delta) = sum r(exp(delta) T)^2 over the correspondences, every term
// evaluated through the whole association (projection, bilinear model lookup
// with its fractional weights, gates decided on real parts), so its
// derivatives include how the looked-up model point and normal move with the
// pose.  The gradient comes from 6 complex-step runs (delta_a = i h), the
// Hessian from 21 bicomplex runs (delta_a on i1, delta_b on i2; a = b carries
// both), exact to rounding at h = 1e-20.
// ---------------------------------------------------------------------------
template <class S>
S icp_energy(const Ctx& X, const Params<S>& P, const Maps<S>& cur, const Maps<S>& model, const Intr<S>& K,
             const M4<S>& Tprev, const M4<S>& T, int64_t* cnt, bool hold) {
  S E(0.0);
  int64_t c = 0;
  for (int i = 0; i < cur.W * cur.H; ++i) {
    S r, J[6];
    if (!icp_residual(X, P, cur, model, K, Tprev, T, i, r, J, hold)) continue;
    E = E + r * r;
    c += 1;
  }
  if (cnt) *cnt = c;
  return E;
}

template <class S> Maps<S> lift_maps(const Maps<double>& M) {
  Maps<S> O;
  O.W = M.W; O.H = M.H; O.valid = M.valid; O.vvalid = M.vvalid; O.Z = M.Z;
  O.V.resize(M.V.size()); O.N.resize(M.N.size());
  for (size_t i = 0; i < M.V.size(); ++i) {
    O.V[i] = V3<S>(S(M.V[i].x), S(M.V[i].y), S(M.V[i].z));
    O.N[i] = V3<S>(S(M.N[i].x), S(M.N[i].y), S(M.N[i].z));
  }
  return O;
}
template <class S> M4<S> lift_pose(const M4<double>& T) {
  M4<S> O;
  for (int k = 0; k < 16; ++k) O.m[k] = S(T.m[k]);
  return O;
}

struct Derivs { double E; double g[6]; double H[21]; int64_t cnt; };

// E, its gradient and Hessian in the left increment delta at delta = 0, for a
// real pose T (real parameters: the configuration's own seed is not applied).
inline Derivs icp_energy_derivs(const Ctx& X, int level, const Maps<double>& cur, const Maps<double>& model,
                                const M4<double>& Tprev, const M4<double>& T, bool hold, int order = 2) {
  const double h = 1e-20;
  Derivs D;
  for (int a = 0; a < 6; ++a) D.g[a] = 0.0;
  for (int k = 0; k < 21; ++k) D.H[k] = 0.0;
  Ctx X0 = X;
  X0.s = OrcSeed{0, -1, -1, 0.0};
  Params<double> P0 = make_params<double>(X0);
  D.E = icp_energy(X0, P0, cur, model, level_intr(P0, X0.c, level), Tprev, T, &D.cnt, hold);
  if (order < 1) return D;
  Maps<cd> curc = lift_maps<cd>(cur), modc = lift_maps<cd>(model);
  for (int a = 0; a < 6; ++a) {
    Ctx Xa = X;
    Xa.s = OrcSeed{1, a, -1, h};
    Params<cd> Pa = make_params<cd>(Xa);
    cd dx[6];
    for (int c = 0; c < 6; ++c) dx[c] = Xa.par<cd>(0.0, c);
    cd E = icp_energy(Xa, Pa, curc, modc, level_intr(Pa, Xa.c, level), lift_pose<cd>(Tprev),
                      mul(se3_exp(dx), lift_pose<cd>(T)), nullptr, hold);
    D.g[a] = E.imag() / h;
  }
  if (order < 2) return D;
  Maps<Bicomplex> curb = lift_maps<Bicomplex>(cur), modb = lift_maps<Bicomplex>(model);
  int k = 0;
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b, ++k) {
      Ctx Xb = X;
      Xb.s = OrcSeed{2, a, b, h};
      Params<Bicomplex> Pb = make_params<Bicomplex>(Xb);
      Bicomplex dx[6];
      for (int c = 0; c < 6; ++c) dx[c] = Xb.par<Bicomplex>(0.0, c);
      Bicomplex E = icp_energy(Xb, Pb, curb, modb, level_intr(Pb, Xb.c, level), lift_pose<Bicomplex>(Tprev),
                               mul(se3_exp(dx), lift_pose<Bicomplex>(T)), nullptr, hold);
      D.H[k] = E.b.imag() / (h * h);
    }
  return D;
}

// One Newton pass: delta = -H^-1 g when the Hessian's LDL^T pivots pass the
// solver's test (positive definite), else the Gauss-Newton step of the same
// pass (classic J, correspondences held fixed).  false: lost.
inline bool newton_step(const Ctx& X, int level, const Maps<double>& cur, const Maps<double>& model,
                        const M4<double>& Tprev, const M4<double>& T, double dx[6], int64_t* cnt, double* r2) {
  // solver 1: correspondences held fixed within the pass; 2: through the association
  Derivs D = icp_energy_derivs(X, level, cur, model, Tprev, T, X.c.solver == 1);
  *cnt = D.cnt;
  *r2 = D.E;
  if (D.cnt < 6) return false;
  double Ah[21], bh[6];
  for (int k = 0; k < 21; ++k) Ah[k] = 0.5 * D.H[k];
  for (int a = 0; a < 6; ++a) bh[a] = 0.5 * D.g[a];
  if (solve6(Ah, bh, dx)) return true;
  Ctx X0 = X;
  X0.s = OrcSeed{0, -1, -1, 0.0};
  Params<double> P0 = make_params<double>(X0);
  Normal<double> G = icp_reduce(X0, P0, cur, model, level_intr(P0, X0.c, level), Tprev, T);
  return solve6(G.A, G.b, dx);
}

// ---------------------------------------------------------------------------
// A6. TSDF fusion (Sec. 4.1 "Surface Update")
// ---------------------------------------------------------------------------
template <class S> struct Volume {
  int dim[3];
  double s;
  std::vector<S> F, W;
  // optional footprint of the raycast (measurement only, never read back by
  // the method): bit 1 = a corner of a marched sample's cell, bit 2 = a corner
  // of a cell evaluated at a hit (the bracket and the six gradient samples)
  uint8_t* touch = nullptr;
};

// depth lookup L(x) for fusion: bilinear over 4 valid taps with the same
// discontinuity rule as the model lookup.  Returns false if unusable.
template <class S>
bool depth_lookup(const std::vector<S>& D, int W, int H, const S& ux, const S& uy, double delta, S& out) {
  double rx = re(ux), ry = re(uy);
  double fx0 = std::floor(rx), fy0 = std::floor(ry);
  if (!(fx0 >= 0.0 && fy0 >= 0.0 && fx0 <= double(W - 2) && fy0 <= double(H - 2))) return false;
  int i0 = int(fx0), j0 = int(fy0);
  int t[4] = {j0 * W + i0, j0 * W + i0 + 1, (j0 + 1) * W + i0, (j0 + 1) * W + i0 + 1};
  for (int k = 0; k < 4; ++k)
    if (!(re(D[t[k]]) > 0.0)) return false;
  int in = int(std::floor(rx + 0.5)), jn = int(std::floor(ry + 0.5));
  int tn = jn * W + in;
  double disc = 0.0;
  for (int k = 0; k < 4; ++k) disc += std::fabs(re(D[t[k]]) - re(D[tn]));
  if (disc >= delta) { out = D[tn]; return true; }
  S a = ux - S(double(i0)), b = uy - S(double(j0));
  S a1 = S(1.0) - a, b1 = S(1.0) - b;
  out = b1 * (a1 * D[t[0]] + a * D[t[1]]) + b * (a1 * D[t[2]] + a * D[t[3]]);
  return true;
}

// Per voxel centre c = (i+1/2)s - L/2 (world origin at the volume centre):
//   x = T^-1 c; u = pi(K x); eta = L(u) - x_z  (eq. bi_interpolate: the
//   ray-length ratio times |t - p| equals x_z at u = pi(K T^-1 p); the sign
//   makes free space positive, as the raycast's crossing test assumes);
//   Psi(eta) = clamp(eta/mu, -1, 1) for eta >= -mu, else no update;
//   F <- (W F + Psi)/(W + 1); W <- min(W + 1, W_cap) (cap taken on a tie).
// Returns 1 if the voxel was updated.
template <class S>
int fuse_voxel(const Ctx& X, const Params<S>& P, const int dim[3], double s, int64_t idx, S& F, S& Wt,
               const std::vector<S>& D, const M4<S>& T) {
  int nx = dim[0], ny = dim[1];
  int i = int(idx % nx), j = int((idx / nx) % ny), k = int(idx / (int64_t(nx) * ny));
  V3<S> c(S((i + 0.5) * s - 0.5 * nx * s), S((j + 0.5) * s - 0.5 * ny * s), S((k + 0.5) * s - 0.5 * dim[2] * s));
  V3<S> x = apply_inv(T, c);
  if (!(re(x.z) > 0.0)) return 0;
  S ux = P.fx * x.x / x.z + P.cx;
  S uy = P.fy * x.y / x.z + P.cy;
  S L;
  if (!depth_lookup(D, X.c.width, X.c.height, ux, uy, X.c.disc_delta, L)) return 0;
  S eta = L - x.z;
  if (re(eta) < -re(P.mu)) return 0;
  S Fd = (re(eta) >= re(P.mu)) ? S(1.0) : eta / P.mu;
  F = (Wt * F + Fd) / (Wt + S(1.0));
  Wt = (re(Wt) + 1.0 < re(P.wcap)) ? Wt + S(1.0) : P.wcap;
  return 1;
}

// ---------------------------------------------------------------------------
// Camera relocalisation objective (Sec. 5.2, eq. of E(T_{g,q})): with a
// reference volume M_r = (F_r, W_r) and a query depth D_q fused at the
// candidate pose T_q, F_q = surface_update(M_r, T_q, D_q) and
// E(T_q) = sum_p (F_r(p) - F_q(p))^2.  A voxel the update leaves alone
// contributes 0; an updated voxel has F_q = (W_r F_r + F_D) / (W_r + 1), so it
// contributes ((F_r - F_D) / (W_r + 1))^2.  Voxels the reference never
// observed (W_r = 0) carry no reference value and are left out.  The update's
// decisions and F_D are those of fuse_voxel (decisions on real parts).
// ---------------------------------------------------------------------------
template <class S>
bool reloc_voxel(const Ctx& X, const Params<S>& P, const int dim[3], double s, int64_t idx, double Fr, double Wr,
                 const std::vector<S>& D, const M4<S>& T, S& contrib) {
  if (!(Wr > 0.0)) return false;
  int nx = dim[0], ny = dim[1];
  int i = int(idx % nx), j = int((idx / nx) % ny), k = int(idx / (int64_t(nx) * ny));
  V3<S> c(S((i + 0.5) * s - 0.5 * nx * s), S((j + 0.5) * s - 0.5 * ny * s), S((k + 0.5) * s - 0.5 * dim[2] * s));
  V3<S> x = apply_inv(T, c);
  if (!(re(x.z) > 0.0)) return false;
  S ux = P.fx * x.x / x.z + P.cx;
  S uy = P.fy * x.y / x.z + P.cy;
  S L;
  if (!depth_lookup(D, X.c.width, X.c.height, ux, uy, X.c.disc_delta, L)) return false;
  S eta = L - x.z;
  if (re(eta) < -re(P.mu)) return false;
  S Fd = (re(eta) >= re(P.mu)) ? S(1.0) : eta / P.mu;
  S d = (S(Fr) - Fd) / S(Wr + 1.0);
  contrib = d * d;
  return true;
}

// E over the whole volume, voxels in index order (the oracle's fixed order)
template <class S>
S reloc_energy(const Ctx& X, const Params<S>& P, const OrcConfig& c, const double* F, const double* W,
               const std::vector<S>& D, const M4<S>& T, int64_t* cnt) {
  int64_t n = int64_t(c.dim[0]) * c.dim[1] * c.dim[2];
  S E(0.0);
  int64_t m = 0;
  for (int64_t v = 0; v < n; ++v) {
    S e;
    if (!reloc_voxel(X, P, c.dim, c.voxel, v, F[v], W[v], D, T, e)) continue;
    E = E + e;
    m += 1;
  }
  if (cnt) *cnt = m;
  return E;
}

// ---------------------------------------------------------------------------
// A7. raycast (Sec. 4.1 "Ray casting", eq. surface_prediction)
// ---------------------------------------------------------------------------
// trilinear F at a world point; valid only if all 8 corners are observed (W>0)
template <class S> bool trilinear(const Volume<S>& Vol, const V3<S>& v, S& out, uint8_t touch_bit = 1) {
  S g[3] = {v.x, v.y, v.z};
  int i0[3];
  S f[3];
  for (int a = 0; a < 3; ++a) {
    S ga = (g[a] + S(0.5 * Vol.dim[a] * Vol.s)) / S(Vol.s) - S(0.5);
    double fl = std::floor(re(ga));
    if (!(fl >= 0.0 && fl <= double(Vol.dim[a] - 2))) return false;
    i0[a] = int(fl);
    f[a] = ga - S(fl);
  }
  int nx = Vol.dim[0], ny = Vol.dim[1];
  if (Vol.touch) {
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          int64_t id = (int64_t(i0[2] + dz) * ny + (i0[1] + dy)) * nx + (i0[0] + dx);
#pragma omp atomic update
          Vol.touch[id] |= touch_bit;
        }
  }
  S c[8];
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        int64_t id = (int64_t(i0[2] + dz) * ny + (i0[1] + dy)) * nx + (i0[0] + dx);
        if (!(re(Vol.W[id]) > 0.0)) return false;
        c[dz * 4 + dy * 2 + dx] = Vol.F[id];
      }
  S fx1 = S(1.0) - f[0], fy1 = S(1.0) - f[1], fz1 = S(1.0) - f[2];
  S c00 = fx1 * c[0] + f[0] * c[1], c10 = fx1 * c[2] + f[0] * c[3];
  S c01 = fx1 * c[4] + f[0] * c[5], c11 = fx1 * c[6] + f[0] * c[7];
  S c0 = fy1 * c00 + f[1] * c10, c1 = fy1 * c01 + f[1] * c11;
  out = fz1 * c0 + f[2] * c1;
  return true;
}

template <class S> struct Hit { bool ok = false; V3<S> V, N; double z = 0.0; };

// Optional real march schedule taken from another run (finite-difference pins
// only): start/end and step sizes come from pose Ts and (mu, fx, fy, cx, cy),
// so a perturbed real run samples at the base run's alphas, which is what the
// complex run does (its alphas are real).
struct Sched { double T[16]; double mu, fx, fy, cx, cy; };

// March the ray o + alpha R K^-1 (u,1) (alpha = camera depth).  The sample
// schedule uses real parts only: half a voxel while the last sample is
// observed and within the truncation band (F < 0.999), else 0.8 mu; from
// max(near, entry) to the exit of the volume shrunk by one voxel.  A crossing
// F_m > 0 > F_{m+1} between two consecutive valid samples is a hit, located by
// alpha0 = alpha_m - dalpha F_m / (F_{m+1} - F_m); a crossing - to + ends the
// ray without a hit; an unobserved sample breaks the pair.  N = normalised
// central-difference gradient of F at +-1 voxel (all six samples valid).
template <class S>
Hit<S> raycast_pixel(const Ctx& X, const Params<S>& P, const Volume<S>& Vol, const M4<S>& T, int x, int y,
                     const Sched* sc = nullptr) {
  Hit<S> H;
  V3<S> dh((S(double(x)) - P.cx) / P.fx, (S(double(y)) - P.cy) / P.fy, S(1.0));
  V3<S> dir = rotate(T, dh);
  V3<S> o(T(0, 3), T(1, 3), T(2, 3));
  double orr[3] = {re(o.x), re(o.y), re(o.z)}, dr[3] = {re(dir.x), re(dir.y), re(dir.z)};
  double dhx = re(dh.x), dhy = re(dh.y), mu = re(P.mu);
  if (sc) {
    dhx = (double(x) - sc->cx) / sc->fx;
    dhy = (double(y) - sc->cy) / sc->fy;
    for (int a = 0; a < 3; ++a) {
      orr[a] = sc->T[a * 4 + 3];
      dr[a] = sc->T[a * 4 + 0] * dhx + sc->T[a * 4 + 1] * dhy + sc->T[a * 4 + 2];
    }
    mu = sc->mu;
  }
  double nrm = std::sqrt(dhx * dhx + dhy * dhy + 1.0);
  double s = Vol.s;
  double tmin = -1e300, tmax = 1e300;
  for (int a = 0; a < 3; ++a) {
    double lo = -0.5 * Vol.dim[a] * s + s, hi = 0.5 * Vol.dim[a] * s - s;
    if (dr[a] != 0.0) {
      double t1 = (lo - orr[a]) / dr[a], t2 = (hi - orr[a]) / dr[a];
      tmin = std::max(tmin, std::min(t1, t2));
      tmax = std::min(tmax, std::max(t1, t2));
    } else if (orr[a] < lo || orr[a] > hi) {
      return H;
    }
  }
  double alpha = std::max(X.c.near_m, tmin);
  bool prev_ok = false;
  double a_prev = 0.0, f_prev = 0.0;
  for (int it = 0; it < 100000 && alpha <= tmax; ++it) {
    V3<S> v = o + S(alpha) * dir;
    S Fs;
    bool ok = trilinear(Vol, v, Fs);
    double f = ok ? re(Fs) : 0.0;
    if (ok && prev_ok) {
      if (f_prev > 0.0 && f < 0.0) {
        // recompute both samples in S and interpolate the crossing
        S F0, F1;
        trilinear(Vol, o + S(a_prev) * dir, F0, 2);
        F1 = Fs;
        if (Vol.touch) trilinear(Vol, v, F1, 2);   // footprint only: same cell, same value
        S a0 = S(a_prev) - S(alpha - a_prev) * F0 / (F1 - F0);
        V3<S> Vg = o + a0 * dir;
        S gr[3];
        for (int a = 0; a < 3; ++a) {
          V3<S> e(S(a == 0 ? s : 0.0), S(a == 1 ? s : 0.0), S(a == 2 ? s : 0.0));
          S fp, fm;
          if (!trilinear(Vol, Vg + e, fp, 2) || !trilinear(Vol, Vg - e, fm, 2)) return H;
          gr[a] = fp - fm;
        }
        V3<S> g(gr[0], gr[1], gr[2]);
        S gg = dot(g, g);
        if (!(re(gg) > 0.0)) return H;
        H.ok = true;
        H.V = Vg;
        H.N = (S(1.0) / sqrt(gg)) * g;
        H.z = re(a0);
        return H;
      }
      if (f_prev < 0.0 && f > 0.0) return H;
    }
    double step = (ok && f < 0.999) ? 0.5 * s / nrm : 0.8 * mu / nrm;
    prev_ok = ok;
    a_prev = alpha;
    f_prev = f;
    alpha = alpha + step;
  }
  return H;
}

template <class S>
Maps<S> raycast(const Ctx& X, const Params<S>& P, const Volume<S>& Vol, const M4<S>& T,
                const Sched* sc = nullptr) {
  Maps<S> M;
  int W = X.c.width, Hh = X.c.height, n = W * Hh;
  M.W = W; M.H = Hh;
  M.V.assign(n, V3<S>()); M.N.assign(n, V3<S>()); M.valid.assign(n, 0); M.vvalid.assign(n, 0); M.Z.assign(n, 0.0);
  // rays are independent: an optional thread split changes nothing
#pragma omp parallel for schedule(dynamic, 4)
  for (int y = 0; y < Hh; ++y)
    for (int x = 0; x < W; ++x) {
      Hit<S> h = raycast_pixel(X, P, Vol, T, x, y, sc);
      if (!h.ok) continue;
      int i = y * W + x;
      M.V[i] = h.V; M.N[i] = h.N; M.Z[i] = h.z; M.valid[i] = 1; M.vvalid[i] = 1;
    }
  return M;
}

// model maps of coarser levels: level-0 maps sampled at (2^l x, 2^l y)
template <class S> Maps<S> subsample(const Maps<S>& M0, int l) {
  Maps<S> M;
  M.W = M0.W >> l; M.H = M0.H >> l;
  int n = M.W * M.H;
  M.V.resize(n); M.N.resize(n); M.valid.resize(n); M.vvalid.resize(n); M.Z.resize(n);
  for (int y = 0; y < M.H; ++y)
    for (int x = 0; x < M.W; ++x) {
      int s = (y << l) * M0.W + (x << l), d = y * M.W + x;
      M.V[d] = M0.V[s]; M.N[d] = M0.N[s]; M.valid[d] = M0.valid[s]; M.vvalid[d] = M0.vvalid[s]; M.Z[d] = M0.Z[s];
    }
  return M;
}

// ---------------------------------------------------------------------------
// A8. frame orchestration (Sec. 4.1 stage order) and trajectory error
// ---------------------------------------------------------------------------
template <class S> struct Measured {
  std::vector<S> Dl[3];
  Maps<S> M[3];
};

template <class S> Measured<S> measure(const Ctx& X, const Params<S>& P, const double* D, const double* Ddot) {
  Measured<S> R;
  R.Dl[0] = bilateral(X, promote_depth<S>(X, D, Ddot));
  int W = X.c.width, H = X.c.height;
  for (int l = 1; l < 3; ++l) {
    R.Dl[l] = pyrdown(X, R.Dl[l - 1], W >> (l - 1), H >> (l - 1));
  }
  for (int l = 0; l < 3; ++l) R.M[l] = vertex_normal(R.Dl[l], level_intr(P, X.c, l));
  return R;
}

struct FrameStats { int32_t lost; int32_t cnt_last; double r2_last; int64_t n_fused; int64_t n_hits; int64_t cnt_sum; };

template <class S> struct State {
  Volume<S> vol;
  Maps<S> model[3];
  M4<S> T, Tprev;   // current (after the last frame) and the one before
  int frame = 0;
  int lost1 = 0, lost2 = 0;   // lost flags of the last frame and the one before
};

// Constant-velocity initial estimate for the ICP of frame k (config init = 1;
// the paper starts from the previous pose): T1 T2^-1 T1 from the poses of
// frames k-1 (T1) and k-2 (T2), used only when both of those frames were
// tracked -- after a lost frame the velocity is unknown and the previous pose
// T1 is the estimate.  The extrapolated rotation R1 R2^T R1 roughly triples any
// departure from orthonormality and each prediction starts from the last, so
// it is brought back by two Newton steps of the polar decomposition,
// R <- 1.5 R - 0.5 R (R^T R) (quadratic convergence to the nearest rotation);
// the translation is left as extrapolated.
template <class S> void polar2(M4<S>& P) {
  for (int it = 0; it < 2; ++it) {
    S G[3][3], N[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) G[r][c] = P(0, r) * P(0, c) + P(1, r) * P(1, c) + P(2, r) * P(2, c);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        N[r][c] = S(1.5) * P(r, c) - S(0.5) * (P(r, 0) * G[0][c] + P(r, 1) * G[1][c] + P(r, 2) * G[2][c]);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) P(r, c) = N[r][c];
  }
}
template <class S> M4<S> const_velocity(const M4<S>& T1, const M4<S>& T2, bool both_tracked) {
  if (!both_tracked) return T1;
  M4<S> P = mul(T1, mul(inverse(T2), T1));
  polar2(P);
  return P;
}

template <class S>
M4<S> track(const Ctx& X, const Params<S>& P, const Measured<S>& meas, const Maps<S> model[3],
            const M4<S>& Tprev, const M4<S>& Tinit, int32_t& lost, Normal<S>* last = nullptr,
            int64_t* cnt_sum = nullptr) {
  M4<S> T = Tinit;
  lost = 0;
  if (cnt_sum) *cnt_sum = 0;
  for (int l = 2; l >= 0 && !lost; --l) {
    Intr<S> K = level_intr(P, X.c, l);
    for (int it = 0; it < X.c.iters[l]; ++it) {
      S dx[6];
      if constexpr (std::is_same<S, double>::value) {
        if (X.c.solver >= 1) {
          // Newton pass with the complex-step gradient and Hessian
          int64_t cnt = 0;
          double r2 = 0.0;
          const bool ok = newton_step(X, l, meas.M[l], model[l], Tprev, T, dx, &cnt, &r2);
          if (last) { last->cnt = cnt; last->r2 = r2; }
          if (cnt_sum) *cnt_sum += cnt;
          if (!ok) { lost = 1; break; }
          for (int a = 0; a < 6; ++a) dx[a] = P.w[l] * dx[a];
          if (X.c.update == 1) {
            T = mul(small_angle(dx), T);
            polar2(T);
          } else {
            T = mul(se3_exp(dx), T);
          }
          continue;
        }
      }
      Normal<S> E = icp_reduce(X, P, meas.M[l], model[l], K, Tprev, T);
      if (last) *last = E;
      if (cnt_sum) *cnt_sum += E.cnt;
      if (E.cnt < 6 || !solve6(E.A, E.b, dx)) { lost = 1; break; }
      for (int a = 0; a < 6; ++a) dx[a] = P.w[l] * dx[a];
      if (X.c.update == 1) {
        // original KinectFusion form: the linearised increment, then the
        // rotation brought back to orthonormal
        T = mul(small_angle(dx), T);
        polar2(T);
      } else {
        T = mul(se3_exp(dx), T);
      }
    }
  }
  if (lost) T = Tinit;
  return T;
}

template <class S>
int64_t fuse(const Ctx& X, const Params<S>& P, Volume<S>& Vol, const std::vector<S>& D, const M4<S>& T) {
  int64_t n = int64_t(Vol.dim[0]) * Vol.dim[1] * Vol.dim[2], cnt = 0;
  // voxels are independent: an optional thread split changes nothing
#pragma omp parallel for schedule(static) reduction(+ : cnt)
  for (int64_t i = 0; i < n; ++i) cnt += fuse_voxel(X, P, Vol.dim, Vol.s, i, Vol.F[i], Vol.W[i], D, T);
  return cnt;
}

template <class S>
void frame_step(const Ctx& X, const Params<S>& P, State<S>& St, const double* D, const double* Ddot,
                FrameStats& fs, const Sched* sc = nullptr) {
  Measured<S> meas = measure(X, P, D, Ddot);
  fs = FrameStats{0, 0, 0.0, 0, 0, 0};
  if (St.frame > 0) {
    M4<S> Tinit = St.T;
    if (X.c.init == 1 && St.frame > 1) Tinit = const_velocity(St.T, St.Tprev, !St.lost1 && !St.lost2);
    Normal<S> last;
    int32_t lost = 0;
    M4<S> T = track(X, P, meas, St.model, St.T, Tinit, lost, &last, &fs.cnt_sum);
    fs.lost = lost; fs.cnt_last = int32_t(last.cnt); fs.r2_last = last.r2;
    St.Tprev = St.T;
    St.T = T;
  }
  St.lost2 = St.lost1;
  St.lost1 = fs.lost;
  if (!fs.lost) fs.n_fused = fuse(X, P, St.vol, meas.Dl[0], St.T);
  St.model[0] = raycast(X, P, St.vol, St.T, sc);
  fs.n_hits = 0;
  for (uint8_t v : St.model[0].valid) fs.n_hits += v;
  St.model[1] = subsample(St.model[0], 1);
  St.model[2] = subsample(St.model[0], 2);
  St.frame += 1;
}

// ---------------------------------------------------------------------------
// F4. X-PointFusion front end (Sec. 4.2): surfel map, 4x4 super-resolution
// index map, one-to-many Gaussian association, confidence-weighted update.
// ---------------------------------------------------------------------------
// Global model points: position v, normal n, radius r, confidence c (all in
// the arithmetic S, so they carry the perturbation's parts) and time stamp t.
template <class S> struct Surfels {
  std::vector<V3<S>> v, n;
  std::vector<S> r, c;
  std::vector<int32_t> t;
  size_t size() const { return v.size(); }
};

template <class S> struct PfState {
  Surfels<S> map;
  Maps<S> model[3];
  M4<S> T, Tprev;
  int frame = 0;
  int lost1 = 0, lost2 = 0;
};

// Real part of a pose.
template <class S> M4<double> re_pose(const M4<S>& T) {
  M4<double> R;
  for (int k = 0; k < 16; ++k) R.m[k] = re(T.m[k]);
  return R;
}
template <class S> V3<double> re_vec(const V3<S>& a) { return V3<double>(re(a.x), re(a.y), re(a.z)); }

// Index map at `sup` x the image resolution (sup = 4 for the association, 1
// for the predicted model maps): every surfel with c >= c_min is projected
// with the real pose, pixel u = pi(K x) with pixel centres at integers, and
// lands in the sub-pixel (floor(sup (u_x + 1/2)), floor(sup (u_y + 1/2)));
// each sub-pixel keeps the surfel nearest to the camera (camera z rounded to
// FP32, ties to the lower index).  -1: empty.
template <class S>
std::vector<int64_t> pf_index_map(const Surfels<S>& M, const M4<S>& T, const Params<S>& P, int W, int H, int sup,
                                  double c_min) {
  const M4<double> Tr = re_pose(T);
  const double fx = re(P.fx), fy = re(P.fy), cx = re(P.cx), cy = re(P.cy);
  const int WS = W * sup, HS = H * sup;
  std::vector<int64_t> idx(size_t(WS) * HS, -1);
  std::vector<float> zb(size_t(WS) * HS, 0.0f);
  for (size_t i = 0; i < M.size(); ++i) {
    if (!(re(M.c[i]) >= c_min)) continue;
    const V3<double> x = apply_inv(Tr, re_vec(M.v[i]));
    if (!(x.z > 0.0)) continue;
    const double ux = fx * x.x / x.z + cx, uy = fy * x.y / x.z + cy;
    const double ax = std::floor(double(sup) * (ux + 0.5)), ay = std::floor(double(sup) * (uy + 0.5));
    if (!(ax >= 0.0 && ay >= 0.0 && ax < double(WS) && ay < double(HS))) continue;
    const size_t q = size_t(ay) * WS + size_t(ax);
    const float zf = float(x.z);
    if (idx[q] < 0 || zf < zb[q]) { idx[q] = int64_t(i); zb[q] = zf; }   // surfels in index order: ties keep the lower
  }
  return idx;
}

// Confidence of a measurement at pixel (x, y) (the PointFusion weight):
// C = exp(-gamma^2 / 0.72), gamma the pixel's radial distance from the
// principal point over the principal point's distance from the image corner
// (0 at the centre, about 1 at the corners).
template <class S> S pf_confidence(const Params<S>& P, int x, int y) {
  const S dx = S(double(x)) - P.cx, dy = S(double(y)) - P.cy;
  const S g2 = (dx * dx + dy * dy) / (P.cx * P.cx + P.cy * P.cy);
  return exp(-g2 / S(0.72));
}

// Surfel radius of a measurement: sqrt(2) z / (f |n_z|), n_z the measured
// normal's camera-z component, its magnitude bounded below by 0.25 (grazing
// views), its sign taken from the real part.
template <class S> S pf_radius(const Params<S>& P, const V3<S>& Vc, const V3<S>& Nc) {
  S nz = re(Nc.z) < 0.0 ? -Nc.z : Nc.z;
  if (re(nz) < 0.25) nz = S(0.25);
  return S(std::sqrt(2.0)) * Vc.z / (P.fx * nz);
}

struct PfCounts { int64_t updated = 0, inserted = 0, dropped = 0; };

// Data association and surface update of frame k at pose T: for each valid
// measured pixel (row-major), the qualified candidates among the surfels of
// its 4x4 block of the index map (rendered before the update) are updated
// with weight w C(u); a pixel with no qualified candidate becomes a new
// surfel, appended in pixel order (up to the capacity).
template <class S>
PfCounts pf_update(const Ctx& X, const Params<S>& P, Surfels<S>& M, const Maps<S>& meas, const M4<S>& T, int k) {
  PfCounts cnt;
  const int W = X.c.width, H = X.c.height, sup = 4;
  const std::vector<int64_t> idx = pf_index_map(M, T, P, W, H, sup, -1e300);
  const M4<double> Tr = re_pose(T);
  const double cos_n = std::cos(X.c.pf_d_norm_deg * M_PI / 180.0);
  const double two_s2 = 2.0 * X.c.pf_sigma * X.c.pf_sigma;
  std::vector<int> fresh;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int u = y * W + x;
      if (!meas.valid[u]) continue;
      const V3<S> Vg = apply(T, meas.V[u]);
      const V3<S> Ng = rotate(T, meas.N[u]);
      const V3<double> vg = re_vec(Vg), ng = re_vec(Ng);
      const double zu = re(meas.V[u].z);
      const S Cu = pf_confidence(P, x, y);
      bool assoc = false;
      for (int sy = 0; sy < sup; ++sy)
        for (int sx = 0; sx < sup; ++sx) {
          const int64_t i = idx[size_t(y * sup + sy) * (W * sup) + size_t(x * sup + sx)];
          if (i < 0) continue;
          // filters, on real parts
          const V3<double> vi = re_vec(M.v[i]), ni = re_vec(M.n[i]);
          const double zi = apply_inv(Tr, vi).z;
          if (!(std::fabs(zi - zu) <= X.c.pf_d_depth)) continue;
          const double nn = std::sqrt(dot(ni, ni));
          if (!(nn > 0.0) || !(dot(ni, ng) >= cos_n * nn)) continue;
          const V3<double> dv = vi - vg;
          if (!(std::sqrt(dot(dv, dv)) <= X.c.pf_d_dist)) continue;
          // one-to-many update with the Gaussian weight of the distance
          const V3<S> d = M.v[i] - Vg;
          const S w = exp(-dot(d, d) / S(two_s2));
          const S a = w * Cu;
          const S den = M.c[i] + a;
          M.v[i] = (S(1.0) / den) * (M.c[i] * M.v[i] + a * Vg);
          M.n[i] = (S(1.0) / den) * (M.c[i] * M.n[i] + a * Ng);
          M.r[i] = (M.c[i] * M.r[i] + a * pf_radius(P, meas.V[u], meas.N[u])) / den;
          M.c[i] = den;
          M.t[i] = k;
          cnt.updated += 1;
          assoc = true;
        }
      if (!assoc) fresh.push_back(u);
    }
  for (int u : fresh) {
    if (M.size() >= size_t(std::max(X.c.pf_capacity, 0))) { cnt.dropped += 1; continue; }
    const int x = u % W, y = u / W;
    M.v.push_back(apply(T, meas.V[u]));
    M.n.push_back(rotate(T, meas.N[u]));
    M.r.push_back(pf_radius(P, meas.V[u], meas.N[u]));
    M.c.push_back(pf_confidence(P, x, y));
    M.t.push_back(k);
    cnt.inserted += 1;
  }
  return cnt;
}

// Predicted model maps at pose T for the next frame's ICP: the nearest
// surfel per pixel among those with c >= c_stable (index map at 1x): V = v,
// N = n / |n|, Z = its camera z (real); levels 1-2 by subsampling.
template <class S> Maps<S> pf_predict(const Ctx& X, const Params<S>& P, const Surfels<S>& M, const M4<S>& T) {
  const int W = X.c.width, H = X.c.height;
  const std::vector<int64_t> idx = pf_index_map(M, T, P, W, H, 1, X.c.pf_c_stable);
  const M4<double> Tr = re_pose(T);
  Maps<S> O;
  O.W = W; O.H = H;
  const int n = W * H;
  O.V.assign(n, V3<S>()); O.N.assign(n, V3<S>()); O.valid.assign(n, 0); O.vvalid.assign(n, 0); O.Z.assign(n, 0.0);
  for (int q = 0; q < n; ++q) {
    const int64_t i = idx[q];
    if (i < 0) continue;
    const S nn = sqrt(dot(M.n[i], M.n[i]));
    if (!(re(nn) > 0.0)) continue;
    O.V[q] = M.v[i];
    O.N[q] = (S(1.0) / nn) * M.n[i];
    O.Z[q] = apply_inv(Tr, re_vec(M.v[i])).z;
    O.valid[q] = 1;
    O.vvalid[q] = 1;
  }
  return O;
}

// One frame of the surfel pipeline: measure, track against the predicted
// maps (as the TSDF path: Sec. 4.2 takes pose estimation from KF), update
// the map (skipped on a lost frame), predict the maps at the new pose.
template <class S>
void pf_frame_step(const Ctx& X, const Params<S>& P, PfState<S>& St, const double* D, const double* Ddot,
                   FrameStats& fs, PfCounts& pc) {
  Measured<S> meas = measure(X, P, D, Ddot);
  fs = FrameStats{0, 0, 0.0, 0, 0, 0};
  pc = PfCounts{};
  if (St.frame > 0) {
    M4<S> Tinit = St.T;
    if (X.c.init == 1 && St.frame > 1) Tinit = const_velocity(St.T, St.Tprev, !St.lost1 && !St.lost2);
    Normal<S> last;
    int32_t lost = 0;
    M4<S> T = track(X, P, meas, St.model, St.T, Tinit, lost, &last, &fs.cnt_sum);
    fs.lost = lost; fs.cnt_last = int32_t(last.cnt); fs.r2_last = last.r2;
    St.Tprev = St.T;
    St.T = T;
  }
  St.lost2 = St.lost1;
  St.lost1 = fs.lost;
  if (!fs.lost) {
    pc = pf_update(X, P, St.map, meas.M[0], St.T, St.frame);
    fs.n_fused = pc.updated;
  }
  St.model[0] = pf_predict(X, P, St.map, St.T);
  for (uint8_t v : St.model[0].valid) fs.n_hits += v;
  St.model[1] = subsample(St.model[0], 1);
  St.model[2] = subsample(St.model[0], 2);
  St.frame += 1;
}

template <class S> M4<S> load_pose(const double* p) {
  M4<S> T;
  for (int i = 0; i < 16; ++i) T.m[i] = get<S>(p + i * NC<S>::n);
  return T;
}
template <class S> void store_pose(double* p, const M4<S>& T) {
  for (int i = 0; i < 16; ++i) put(p + i * NC<S>::n, T.m[i]);
}
template <class S> M4<S> real_pose(const double* p) {
  M4<S> T;
  for (int i = 0; i < 16; ++i) T.m[i] = S(p[i]);
  return T;
}

// initial pose with the pose-seed directions applied on the left: exp(i h e_d) T0
template <class S> M4<S> seeded_initial_pose(const Ctx& X, const double* T0) {
  S xi[6];
  for (int a = 0; a < 6; ++a) xi[a] = X.par<S>(0.0, P_PHI_X + a);
  return mul(se3_exp(xi), real_pose<S>(T0));
}

template <class S> void state_init(const Ctx& X, State<S>& St) {
  for (int a = 0; a < 3; ++a) St.vol.dim[a] = X.c.dim[a];
  St.vol.s = X.c.voxel;
  int64_t n = int64_t(X.c.dim[0]) * X.c.dim[1] * X.c.dim[2];
  St.vol.F.assign(n, S(0.0));
  St.vol.W.assign(n, S(0.0));
}

// ---------------------------------------------------------------------------
// map <-> flat array helpers for the C interface
// ---------------------------------------------------------------------------
template <class S> void maps_out(const Maps<S>& M, double* V, double* N, double* Z, uint8_t* valid) {
  const int nc = NC<S>::n;
  int n = M.W * M.H;
  for (int i = 0; i < n; ++i) {
    if (V) { put(V + (i * 3 + 0) * nc, M.V[i].x); put(V + (i * 3 + 1) * nc, M.V[i].y); put(V + (i * 3 + 2) * nc, M.V[i].z); }
    if (N) { put(N + (i * 3 + 0) * nc, M.N[i].x); put(N + (i * 3 + 1) * nc, M.N[i].y); put(N + (i * 3 + 2) * nc, M.N[i].z); }
    if (Z && !M.Z.empty()) Z[i] = M.Z[i];
    if (valid) valid[i] = M.valid[i];
  }
}
template <class S> Maps<S> maps_in(int W, int H, const double* V, const double* N, const double* Z, const uint8_t* valid) {
  const int nc = NC<S>::n;
  Maps<S> M;
  M.W = W; M.H = H;
  int n = W * H;
  M.V.resize(n); M.N.resize(n); M.valid.resize(n); M.vvalid.resize(n); M.Z.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    M.V[i] = V3<S>(get<S>(V + (i * 3 + 0) * nc), get<S>(V + (i * 3 + 1) * nc), get<S>(V + (i * 3 + 2) * nc));
    M.N[i] = V3<S>(get<S>(N + (i * 3 + 0) * nc), get<S>(N + (i * 3 + 1) * nc), get<S>(N + (i * 3 + 2) * nc));
    if (Z) M.Z[i] = Z[i];
    M.valid[i] = valid[i];
    M.vvalid[i] = valid[i];
  }
  return M;
}
template <class S> void vol_in(Volume<S>& V, const double* F, const double* W) {
  const int nc = NC<S>::n;
  int64_t n = V.F.size();
  for (int64_t i = 0; i < n; ++i) { V.F[i] = get<S>(F + i * nc); V.W[i] = get<S>(W + i * nc); }
}
template <class S> void vol_out(const Volume<S>& V, double* F, double* W) {
  const int nc = NC<S>::n;
  int64_t n = V.F.size();
  for (int64_t i = 0; i < n; ++i) {
    if (F) put(F + i * nc, V.F[i]);
    if (W) put(W + i * nc, V.W[i]);
  }
}

// listed voxels / pixels (threads optional; entries are independent)
template <class S>
int64_t fuse_list(const Ctx& X, const Params<S>& P, const OrcConfig* c, double* F, double* Wt,
                  const std::vector<S>& D, const M4<S>& Tp, const int64_t* idx, int64_t n_idx) {
  const int nc = NC<S>::n;
  int64_t count = 0;
#pragma omp parallel for schedule(static) reduction(+ : count)
  for (int64_t q = 0; q < n_idx; ++q) {
    S f = get<S>(F + q * nc), w = get<S>(Wt + q * nc);
    count += fuse_voxel(X, P, c->dim, c->voxel, idx[q], f, w, D, Tp);
    put(F + q * nc, f);
    put(Wt + q * nc, w);
  }
  return count;
}

template <class S>
void raycast_list(const Ctx& X, const Params<S>& P, const Volume<S>& Vol, const M4<S>& Tp, int width,
                  const int32_t* pix, int npx, const Sched* sc, double* V_out, double* N_out, double* Z_out,
                  uint8_t* valid_out) {
  const int nc = NC<S>::n;
#pragma omp parallel for schedule(dynamic, 64)
  for (int q = 0; q < npx; ++q) {
    int id = pix ? pix[q] : q;
    Hit<S> h = raycast_pixel(X, P, Vol, Tp, id % width, id / width, sc);
    V3<S> V = h.ok ? h.V : V3<S>(), N = h.ok ? h.N : V3<S>();
    put(V_out + (q * 3 + 0) * nc, V.x); put(V_out + (q * 3 + 1) * nc, V.y); put(V_out + (q * 3 + 2) * nc, V.z);
    put(N_out + (q * 3 + 0) * nc, N.x); put(N_out + (q * 3 + 1) * nc, N.y); put(N_out + (q * 3 + 2) * nc, N.z);
    Z_out[q] = h.ok ? h.z : 0.0;
    valid_out[q] = h.ok ? 1 : 0;
  }
}

}  // namespace orc

// ===========================================================================
// C interface.  ncomp = 1 (real), 2 (complex) or 4 (bicomplex) doubles per
// scalar, chosen by seed->kind = 0, 1, 2.  Arrays are row-major; images H x W,
// 3-vector maps H x W x 3 x ncomp, poses 16 x ncomp (row-major 4x4,
// camera-to-world), volumes x-fastest (i + nx (j + ny k)).
// ===========================================================================
using namespace orc;

#define ORC_DISPATCH(seed, ...)                                  \
  do {                                                           \
    if ((seed)->kind == 0) { typedef double S; __VA_ARGS__; }    \
    else if ((seed)->kind == 1) { typedef cd S; __VA_ARGS__; }   \
    else { typedef Bicomplex S; __VA_ARGS__; }                   \
  } while (0)

extern "C" {

int orc_ncomp(const OrcSeed* s) { return s->kind == 0 ? 1 : (s->kind == 1 ? 2 : 4); }

// Threads for the per-voxel and per-ray loops (default 1; results do not depend on it).
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n < 1 ? 1 : n);
#else
  (void)n;
#endif
}

// SE(3) exponential of a 6-vector of scalars.
void orc_se3_exp(const OrcSeed* seed, const double* xi, double* T) {
  ORC_DISPATCH(seed, {
    S x[6];
    for (int a = 0; a < 6; ++a) x[a] = get<S>(xi + a * NC<S>::n);
    store_pose(T, se3_exp(x));
  });
}

// Pose increment of the original KinectFusion form: the small-angle transform
// of eq. icp_approx composed with T (16 x ncomp each), then two polar steps
// on the rotation.  out: 16 x ncomp.
void orc_small_angle_update(const OrcSeed* seed, const double* xi, const double* T, double* out) {
  ORC_DISPATCH(seed, {
    S x[6];
    for (int a = 0; a < 6; ++a) x[a] = get<S>(xi + a * NC<S>::n);
    M4<S> P = mul(small_angle(x), load_pose<S>(T));
    polar2(P);
    store_pose(out, P);
  });
}

// Newton ICP objective of one pass at level `level` (real run): E = sum r^2 at
// pose T against the model maps of that level (projection reference Tprev),
// with the correspondences held fixed (through 0) or differentiated through
// the association (through 1),
// its gradient and Hessian in the left increment (order 0: E only, 1: and the
// gradient, 2: and the Hessian; the others are returned as 0).  out[29]: E,
// g[6], H (21, upper triangle row-major), correspondence count.
void orc_icp_energy(const OrcConfig* c, int level, const double* Vc, const double* Nc, const uint8_t* validc,
                    const double* Vm, const double* Nm, const double* Zm, const uint8_t* validm,
                    const double* Tprev, const double* T, int through, int order, double* out) {
  OrcSeed s0{0, -1, -1, 0.0};
  Ctx X{*c, s0};
  Params<double> P = make_params<double>(X);
  Intr<double> K = level_intr(P, X.c, level);
  Maps<double> cur = maps_in<double>(K.W, K.H, Vc, Nc, nullptr, validc);
  Maps<double> mod = maps_in<double>(K.W, K.H, Vm, Nm, Zm, validm);
  Derivs D = icp_energy_derivs(X, level, cur, mod, load_pose<double>(Tprev), load_pose<double>(T), through == 0, order);
  out[0] = D.E;
  for (int a = 0; a < 6; ++a) out[1 + a] = D.g[a];
  for (int k = 0; k < 21; ++k) out[7 + k] = D.H[k];
  out[28] = double(D.cnt);
}

// Relocalisation objective at the real pose T: reference volume F, W (real,
// x-fastest), the query's filtered level-0 depth Df (real, H x W).  E, its
// gradient and Hessian in the left increment exp(delta) T from 6 complex-step
// and 21 bicomplex evaluations of the whole sum (order 0 / 1: E only / and the
// gradient; the rest returned as 0).  out[29]: E, g[6], H (21, upper triangle
// row-major, order phi then rho), number of contributing voxels.
void orc_reloc_energy(const OrcConfig* c, const double* F, const double* W, const double* Df, const double* T,
                      int order, double* out) {
  const double h = 1e-20;
  const int n = c->width * c->height;
  OrcSeed s0{0, -1, -1, 0.0};
  Ctx X0{*c, s0};
  Params<double> P0 = make_params<double>(X0);
  std::vector<double> D(Df, Df + n);
  M4<double> T0 = load_pose<double>(T);
  int64_t cnt = 0;
  for (int k = 0; k < 29; ++k) out[k] = 0.0;
  out[0] = reloc_energy(X0, P0, *c, F, W, D, T0, &cnt);
  out[28] = double(cnt);
  if (order >= 1) {
    std::vector<cd> Dc(D.begin(), D.end());
    for (int a = 0; a < 6; ++a) {
      Ctx Xa{*c, OrcSeed{1, a, -1, h}};
      Params<cd> Pa = make_params<cd>(Xa);
      cd dx[6];
      for (int q = 0; q < 6; ++q) dx[q] = Xa.par<cd>(0.0, q);
      cd E = reloc_energy(Xa, Pa, *c, F, W, Dc, mul(se3_exp(dx), lift_pose<cd>(T0)), nullptr);
      out[1 + a] = E.imag() / h;
    }
  }
  if (order >= 2) {
    std::vector<Bicomplex> Db(n);
    for (int i = 0; i < n; ++i) Db[i] = Bicomplex(D[i]);
    int k = 0;
    for (int a = 0; a < 6; ++a)
      for (int b = a; b < 6; ++b, ++k) {
        Ctx Xb{*c, OrcSeed{2, a, b, h}};
        Params<Bicomplex> Pb = make_params<Bicomplex>(Xb);
        Bicomplex dx[6];
        for (int q = 0; q < 6; ++q) dx[q] = Xb.par<Bicomplex>(0.0, q);
        Bicomplex E = reloc_energy(Xb, Pb, *c, F, W, Db, mul(se3_exp(dx), lift_pose<Bicomplex>(T0)), nullptr);
        out[7 + k] = E.b.imag() / (h * h);
      }
  }
}

// Surface measurement of one frame: filtered depth per level and V/N maps.
// depth_out: 3 levels concatenated (sizes W_l*H_l), V/N likewise x3xncomp, valid per level.
void orc_measure(const OrcConfig* c, const OrcSeed* seed, const double* depth, const double* depth_dot,
                 double* depth_out, double* V_out, double* N_out, uint8_t* valid_out) {
  Ctx X{*c, *seed};
  ORC_DISPATCH(seed, {
    Params<S> P = make_params<S>(X);
    Measured<S> m = measure(X, P, depth, depth_dot);
    size_t off = 0;
    for (int l = 0; l < 3; ++l) {
      int n = m.M[l].W * m.M[l].H;
      for (int i = 0; i < n; ++i) put(depth_out + (off + i) * NC<S>::n, m.Dl[l][i]);
      maps_out(m.M[l], V_out + off * 3 * NC<S>::n, N_out + off * 3 * NC<S>::n, nullptr, valid_out + off);
      off += n;
    }
  });
}

// One association + reduction pass at level l.  cur/model maps are given for
// that level; model Z is the real model depth.  Out: A[21], b[6] (x ncomp), cnt, r2.
void orc_icp_reduce(const OrcConfig* c, const OrcSeed* seed, int level,
                    const double* Vc, const double* Nc, const uint8_t* validc,
                    const double* Vm, const double* Nm, const double* Zm, const uint8_t* validm,
                    const double* Tprev, const double* T, double* A_out, double* b_out,
                    int64_t* cnt, double* r2) {
  Ctx X{*c, *seed};
  ORC_DISPATCH(seed, {
    Params<S> P = make_params<S>(X);
    Intr<S> K = level_intr(P, X.c, level);
    Maps<S> cur = maps_in<S>(K.W, K.H, Vc, Nc, nullptr, validc);
    Maps<S> mod = maps_in<S>(K.W, K.H, Vm, Nm, Zm, validm);
    Normal<S> E = icp_reduce(X, P, cur, mod, K, load_pose<S>(Tprev), load_pose<S>(T));
    for (int k = 0; k < 21; ++k) put(A_out + k * NC<S>::n, E.A[k]);
    for (int k = 0; k < 6; ++k) put(b_out + k * NC<S>::n, E.b[k]);
    *cnt = E.cnt;
    *r2 = E.r2;
  });
}

// delta = -w A^-1 b; returns 0 ok, 1 lost
int orc_solve(const OrcSeed* seed, const double* A, const double* b, const double* w, double* delta) {
  int rc = 0;
  ORC_DISPATCH(seed, {
    S Au[21], bb[6], x[6];
    for (int k = 0; k < 21; ++k) Au[k] = get<S>(A + k * NC<S>::n);
    for (int k = 0; k < 6; ++k) bb[k] = get<S>(b + k * NC<S>::n);
    if (!solve6(Au, bb, x)) { rc = 1; }
    else {
      S ww = get<S>(w);
      for (int k = 0; k < 6; ++k) put(delta + k * NC<S>::n, ww * x[k]);
    }
  });
  return rc;
}

// Fusion of one frame into (F, W) (in/out, x-fastest, ncomp per scalar) with
// the filtered level-0 depth Df (H x W x ncomp) at pose T.  If idx != NULL only
// the n_idx listed voxels are processed (F, W then hold just those voxels, in
// list order).  Returns the number of updated voxels.
int64_t orc_fuse(const OrcConfig* c, const OrcSeed* seed, double* F, double* Wt, const double* Df,
                 const double* T, const int64_t* idx, int64_t n_idx) {
  Ctx X{*c, *seed};
  int64_t count = 0;
  ORC_DISPATCH(seed, {
    const int nc = NC<S>::n;
    Params<S> P = make_params<S>(X);
    int n = c->width * c->height;
    std::vector<S> D(n);
    for (int i = 0; i < n; ++i) D[i] = get<S>(Df + i * nc);
    M4<S> Tp = load_pose<S>(T);
    if (idx) {
      count = fuse_list<S>(X, P, c, F, Wt, D, Tp, idx, n_idx);
    } else {
      Volume<S> Vol;
      for (int a = 0; a < 3; ++a) Vol.dim[a] = c->dim[a];
      Vol.s = c->voxel;
      int64_t nv = int64_t(c->dim[0]) * c->dim[1] * c->dim[2];
      Vol.F.resize(nv); Vol.W.resize(nv);
      vol_in(Vol, F, Wt);
      count = fuse(X, P, Vol, D, Tp);
      vol_out(Vol, F, Wt);
    }
  });
  return count;
}

// Decision margins of fusion for the listed voxels (measurement of mask
// mismatches only): out[q] = re(eta) + re(mu), the distance of the update test
// eta >= -mu from its threshold, for voxels whose projection and depth taps
// are usable; NaN for voxels decided before that test (behind the camera,
// outside the image, an invalid tap).
void orc_fuse_margin(const OrcConfig* c, const OrcSeed* seed, const double* Df, const double* T,
                     const int64_t* idx, int64_t n_idx, double* out) {
  Ctx X{*c, *seed};
  ORC_DISPATCH(seed, {
    const int nc = NC<S>::n;
    Params<S> P = make_params<S>(X);
    int n = c->width * c->height;
    std::vector<S> D(n);
    for (int i = 0; i < n; ++i) D[i] = get<S>(Df + i * nc);
    M4<S> Tp = load_pose<S>(T);
    int nx = c->dim[0], ny = c->dim[1];
    double sv = c->voxel;
    for (int64_t q = 0; q < n_idx; ++q) {
      int64_t id = idx[q];
      int i = int(id % nx), j = int((id / nx) % ny), k = int(id / (int64_t(nx) * ny));
      V3<S> ctr(S((i + 0.5) * sv - 0.5 * nx * sv), S((j + 0.5) * sv - 0.5 * ny * sv),
                S((k + 0.5) * sv - 0.5 * c->dim[2] * sv));
      V3<S> x = apply_inv(Tp, ctr);
      out[q] = std::nan("");
      if (!(re(x.z) > 0.0)) continue;
      S ux = P.fx * x.x / x.z + P.cx;
      S uy = P.fy * x.y / x.z + P.cy;
      S L;
      if (!depth_lookup(D, c->width, c->height, ux, uy, c->disc_delta, L)) continue;
      out[q] = re(L - x.z) + re(P.mu);
    }
  });
}

// Raycast of (F, W) at pose T into level-0 model maps.  If pix != NULL only
// the n_pix listed pixels (y*W + x) are cast and the outputs hold them in list
// order; otherwise all pixels.
void orc_raycast(const OrcConfig* c, const OrcSeed* seed, const double* F, const double* Wt, const double* T,
                 const int32_t* pix, int32_t n_pix, double* V_out, double* N_out, double* Z_out,
                 uint8_t* valid_out, const double* sched_pose, const double* sched_params) {
  Ctx X{*c, *seed};
  ORC_DISPATCH(seed, {
    const int nc = NC<S>::n;
    Params<S> P = make_params<S>(X);
    Volume<S> Vol;
    for (int a = 0; a < 3; ++a) Vol.dim[a] = c->dim[a];
    Vol.s = c->voxel;
    int64_t nv = int64_t(c->dim[0]) * c->dim[1] * c->dim[2];
    Vol.F.resize(nv); Vol.W.resize(nv);
    vol_in(Vol, F, Wt);
    M4<S> Tp = load_pose<S>(T);
    Sched sc;
    if (sched_pose) {
      for (int i = 0; i < 16; ++i) sc.T[i] = sched_pose[i];
      sc.mu = sched_params[0]; sc.fx = sched_params[1]; sc.fy = sched_params[2];
      sc.cx = sched_params[3]; sc.cy = sched_params[4];
    }
    int npx = pix ? n_pix : c->width * c->height;
    raycast_list<S>(X, P, Vol, Tp, c->width, pix, npx, sched_pose ? &sc : nullptr, V_out, N_out, Z_out, valid_out);
  });
}

// Tracking of one frame (measure + multi-level ICP) against level-0 model maps
// (sub-sampled here for levels 1, 2).  Returns lost (0/1); T_out = final pose.
int orc_track(const OrcConfig* c, const OrcSeed* seed, const double* depth, const double* depth_dot,
              const double* Vm, const double* Nm, const double* Zm, const uint8_t* validm,
              const double* Tprev, const double* Tinit, double* T_out, int64_t* cnt_last, double* r2_last) {
  Ctx X{*c, *seed};
  int32_t lost = 0;
  ORC_DISPATCH(seed, {
    Params<S> P = make_params<S>(X);
    Measured<S> meas = measure(X, P, depth, depth_dot);
    Maps<S> model[3];
    model[0] = maps_in<S>(c->width, c->height, Vm, Nm, Zm, validm);
    model[1] = subsample(model[0], 1);
    model[2] = subsample(model[0], 2);
    Normal<S> last;
    M4<S> T = track(X, P, meas, model, load_pose<S>(Tprev), load_pose<S>(Tinit), lost, &last);
    store_pose(T_out, T);
    if (cnt_last) *cnt_last = last.cnt;
    if (r2_last) *r2_last = last.r2;
  });
  return lost;
}

// Constant-velocity initial estimate from the poses of the last two frames
// (T1 previous, T2 the one before; 16 x ncomp each) and whether both were
// tracked.  out: 16 x ncomp.
void orc_const_vel(const OrcSeed* seed, const double* T1, const double* T2, int32_t both_tracked, double* out) {
  ORC_DISPATCH(seed, {
    store_pose(out, const_velocity(load_pose<S>(T1), load_pose<S>(T2), both_tracked != 0));
  });
}

// One frame step (frame index `frame` >= 1) from a given state, the step the
// sequence runs: measure, track against the previous frame's level-0 model
// maps (levels 1, 2 sub-sampled), fuse unless lost, raycast.  In/out: F, Wt
// (x-fastest volume, ncomp per scalar); Vm, Nm (H x W x 3 x ncomp), Zm, validm
// (level-0 model maps of the previous frame, replaced by this frame's); T1, T2
// (poses of the last two frames, replaced by this frame's and the previous);
// lost12[2] (lost flags of the last two frames, shifted likewise).
// stats_out[6] as in orc_run_sequence.  touch (optional, one byte per voxel,
// OR-ed): the raycast's footprint, bit 1 marched cells, bit 2 cells at hits.
void orc_frame_step(const OrcConfig* c, const OrcSeed* seed, int32_t frame, const double* depth,
                    const double* depth_dot, double* F, double* Wt, double* Vm, double* Nm, double* Zm,
                    uint8_t* validm, double* T1, double* T2, int32_t* lost12, double* stats_out,
                    uint8_t* touch) {
  Ctx X{*c, *seed};
  ORC_DISPATCH(seed, {
    Params<S> P = make_params<S>(X);
    State<S> St;
    state_init(X, St);
    vol_in(St.vol, F, Wt);
    St.model[0] = maps_in<S>(c->width, c->height, Vm, Nm, Zm, validm);
    St.model[1] = subsample(St.model[0], 1);
    St.model[2] = subsample(St.model[0], 2);
    St.T = load_pose<S>(T1);
    St.Tprev = load_pose<S>(T2);
    St.frame = frame;
    St.lost1 = lost12[0];
    St.lost2 = lost12[1];
    St.vol.touch = touch;
    FrameStats fs;
    frame_step(X, P, St, depth, depth_dot, fs);
    vol_out(St.vol, F, Wt);
    maps_out(St.model[0], Vm, Nm, Zm, validm);
    store_pose(T1, St.T);
    store_pose(T2, St.Tprev);
    lost12[0] = St.lost1;
    lost12[1] = St.lost2;
    if (stats_out) {
      stats_out[0] = fs.lost; stats_out[1] = fs.cnt_last; stats_out[2] = fs.r2_last;
      stats_out[3] = double(fs.n_fused); stats_out[4] = double(fs.n_hits); stats_out[5] = double(fs.cnt_sum);
    }
  });
}

// One frame of the surfel pipeline (X-PointFusion front end) from a loaded
// state, written back.  Surfels (capacity c->pf_capacity, *count in use):
// sv, sn [cap][3][nc], sr, sc [cap][nc], st [cap]; model maps of level 0 as
// in orc_frame_step; T1, T2 the poses of the last two frames; lost12 their
// lost flags.  stats_out (6, optional) as orc_frame_step's, with the number
// of surfel updates in place of fused voxels; pf_out (3, optional): updated,
// inserted, dropped (capacity).
void orc_pf_frame_step(const OrcConfig* c, const OrcSeed* seed, int32_t frame, const double* depth,
                       const double* depth_dot, double* sv, double* sn, double* sr, double* sc, int32_t* st,
                       int64_t* count, double* Vm, double* Nm, double* Zm, uint8_t* validm, double* T1, double* T2,
                       int32_t* lost12, double* stats_out, int64_t* pf_out) {
  Ctx X{*c, *seed};
  ORC_DISPATCH(seed, {
    const int nc = NC<S>::n;
    Params<S> P = make_params<S>(X);
    PfState<S> St;
    const int64_t n = *count;
    St.map.v.resize(n); St.map.n.resize(n); St.map.r.resize(n); St.map.c.resize(n); St.map.t.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      St.map.v[i] = V3<S>(get<S>(sv + (i * 3 + 0) * nc), get<S>(sv + (i * 3 + 1) * nc), get<S>(sv + (i * 3 + 2) * nc));
      St.map.n[i] = V3<S>(get<S>(sn + (i * 3 + 0) * nc), get<S>(sn + (i * 3 + 1) * nc), get<S>(sn + (i * 3 + 2) * nc));
      St.map.r[i] = get<S>(sr + i * nc);
      St.map.c[i] = get<S>(sc + i * nc);
      St.map.t[i] = st[i];
    }
    St.model[0] = maps_in<S>(c->width, c->height, Vm, Nm, Zm, validm);
    St.model[1] = subsample(St.model[0], 1);
    St.model[2] = subsample(St.model[0], 2);
    St.T = load_pose<S>(T1);
    St.Tprev = load_pose<S>(T2);
    St.frame = frame;
    St.lost1 = lost12[0];
    St.lost2 = lost12[1];
    FrameStats fs;
    PfCounts pc;
    pf_frame_step(X, P, St, depth, depth_dot, fs, pc);
    const int64_t m = int64_t(St.map.size());
    for (int64_t i = 0; i < m; ++i) {
      put(sv + (i * 3 + 0) * nc, St.map.v[i].x); put(sv + (i * 3 + 1) * nc, St.map.v[i].y);
      put(sv + (i * 3 + 2) * nc, St.map.v[i].z);
      put(sn + (i * 3 + 0) * nc, St.map.n[i].x); put(sn + (i * 3 + 1) * nc, St.map.n[i].y);
      put(sn + (i * 3 + 2) * nc, St.map.n[i].z);
      put(sr + i * nc, St.map.r[i]);
      put(sc + i * nc, St.map.c[i]);
      st[i] = St.map.t[i];
    }
    *count = m;
    maps_out(St.model[0], Vm, Nm, Zm, validm);
    store_pose(T1, St.T);
    store_pose(T2, St.Tprev);
    lost12[0] = St.lost1;
    lost12[1] = St.lost2;
    if (stats_out) {
      stats_out[0] = fs.lost; stats_out[1] = fs.cnt_last; stats_out[2] = fs.r2_last;
      stats_out[3] = double(fs.n_fused); stats_out[4] = double(fs.n_hits); stats_out[5] = double(fs.cnt_sum);
    }
    if (pf_out) { pf_out[0] = pc.updated; pf_out[1] = pc.inserted; pf_out[2] = pc.dropped; }
  });
}

// Whole surfel sequence: frame 0 at exp(seed) T0 (real 4x4), then
// track / update / predict per frame.  depths (and depth_dots or NULL):
// n_frames x H x W.  poses_out: n_frames x 16 x nc; stats_out (optional):
// n_frames x 6 as orc_pf_frame_step's; pf_out (optional): n_frames x 3.
// The final surfels are written to sv, sn, sr, sc, st (capacity
// c->pf_capacity) with their number in *count.
void orc_pf_run_sequence(const OrcConfig* c, const OrcSeed* seed, int32_t n_frames, const double* depths,
                         const double* depth_dots, const double* T0, double* poses_out, double* stats_out,
                         int64_t* pf_out, double* sv, double* sn, double* sr, double* sc, int32_t* st, int64_t* count) {
  Ctx X{*c, *seed};
  ORC_DISPATCH(seed, {
    const int nc = NC<S>::n;
    Params<S> P = make_params<S>(X);
    PfState<S> St;
    St.T = seeded_initial_pose<S>(X, T0);
    St.Tprev = St.T;
    const size_t npx = size_t(c->width) * c->height;
    for (int f = 0; f < n_frames; ++f) {
      FrameStats fs;
      PfCounts pc;
      pf_frame_step(X, P, St, depths + f * npx, depth_dots ? depth_dots + f * npx : nullptr, fs, pc);
      store_pose(poses_out + size_t(f) * 16 * nc, St.T);
      if (stats_out) {
        double* o = stats_out + size_t(f) * 6;
        o[0] = fs.lost; o[1] = fs.cnt_last; o[2] = fs.r2_last; o[3] = double(fs.n_fused);
        o[4] = double(fs.n_hits); o[5] = double(fs.cnt_sum);
      }
      if (pf_out) {
        int64_t* o = pf_out + size_t(f) * 3;
        o[0] = pc.updated; o[1] = pc.inserted; o[2] = pc.dropped;
      }
    }
    const int64_t m = int64_t(St.map.size());
    for (int64_t i = 0; i < m; ++i) {
      put(sv + (i * 3 + 0) * nc, St.map.v[i].x); put(sv + (i * 3 + 1) * nc, St.map.v[i].y);
      put(sv + (i * 3 + 2) * nc, St.map.v[i].z);
      put(sn + (i * 3 + 0) * nc, St.map.n[i].x); put(sn + (i * 3 + 1) * nc, St.map.n[i].y);
      put(sn + (i * 3 + 2) * nc, St.map.n[i].z);
      put(sr + i * nc, St.map.r[i]);
      put(sc + i * nc, St.map.c[i]);
      st[i] = St.map.t[i];
    }
    *count = m;
  });
}

// Input parts of the learned initialiser (real): the level-2 filtered depth
// D2 ((H/4) x (W/4)) reduced once more with the pyramid's gated binomial
// (level 3), and the level-0 model maps sampled at (8x, 8y): hit depth Zm
// and the world normal Nm rotated into the camera frame of the pose T
// (R^T n); invalid model pixels give 0.  depth_out: (H/8) x (W/8);
// model_out: 4 planes of (H/8) x (W/8) (depth, n_x, n_y, n_z), FP32 values.
void orc_cnn_parts(const OrcConfig* c, const double* D2, const double* Nm, const double* Zm, const uint8_t* validm,
                   const double* T, float* depth_out, float* model_out) {
  OrcSeed s0{0, -1, -1, 0.0};
  Ctx X{*c, s0};
  const int W2 = c->width / 4, H2 = c->height / 4, W3 = c->width / 8, H3 = c->height / 8;
  std::vector<double> d2(D2, D2 + size_t(W2) * H2);
  std::vector<double> d3 = pyrdown(X, d2, W2, H2);
  const M4<double> P = load_pose<double>(T);
  const int n3 = W3 * H3;
  for (int y = 0; y < H3; ++y)
    for (int x = 0; x < W3; ++x) {
      const int o = y * W3 + x;
      depth_out[o] = float(d3[size_t(y) * (W2 / 2) + x]);
      const size_t q = size_t(8 * y) * c->width + 8 * x;
      float z = 0.f, nx = 0.f, ny = 0.f, nz = 0.f;
      if (validm[q]) {
        const double n0 = Nm[q * 3 + 0], n1 = Nm[q * 3 + 1], n2 = Nm[q * 3 + 2];
        z = float(Zm[q]);
        nx = float(P(0, 0) * n0 + P(1, 0) * n1 + P(2, 0) * n2);   // R^T n
        ny = float(P(0, 1) * n0 + P(1, 1) * n1 + P(2, 1) * n2);
        nz = float(P(0, 2) * n0 + P(1, 2) * n1 + P(2, 2) * n2);
      }
      model_out[o] = z;
      model_out[n3 + o] = nx;
      model_out[2 * n3 + o] = ny;
      model_out[3 * n3 + o] = nz;
    }
}

// The index map of the surfels (real positions sv [count][3][nc], confidences
// sc [count][nc]) at the real pose T, `sup` x the image resolution, over the
// surfels with c >= c_min: idx_out [sup H][sup W], -1 where empty.
void orc_pf_index_map(const OrcConfig* c, const double* sv, const double* sc, int64_t count, const double* T,
                      int32_t sup, double c_min, int64_t* idx_out) {
  OrcSeed s0{0, -1, -1, 0.0};
  Ctx X{*c, s0};
  Params<double> P = make_params<double>(X);
  Surfels<double> M;
  M.v.resize(count); M.c.resize(count);
  for (int64_t i = 0; i < count; ++i) {
    M.v[i] = V3<double>(sv[i * 3 + 0], sv[i * 3 + 1], sv[i * 3 + 2]);
    M.c[i] = sc[i];
  }
  std::vector<int64_t> idx = pf_index_map(M, load_pose<double>(T), P, c->width, c->height, sup, c_min);
  std::memcpy(idx_out, idx.data(), idx.size() * sizeof(int64_t));
}

// Footprint of the raycast of (F, W) at pose T (one byte per voxel, OR-ed):
// bit 1 = a corner of a marched sample's cell, bit 2 = a corner of a cell
// evaluated at a hit.  Returns the number of hits.
int64_t orc_raycast_footprint(const OrcConfig* c, const OrcSeed* seed, const double* F, const double* Wt,
                              const double* T, uint8_t* touch) {
  Ctx X{*c, *seed};
  int64_t hits = 0;
  ORC_DISPATCH(seed, {
    Params<S> P = make_params<S>(X);
    Volume<S> Vol;
    for (int a = 0; a < 3; ++a) Vol.dim[a] = c->dim[a];
    Vol.s = c->voxel;
    int64_t nv = int64_t(c->dim[0]) * c->dim[1] * c->dim[2];
    Vol.F.resize(nv); Vol.W.resize(nv);
    vol_in(Vol, F, Wt);
    Vol.touch = touch;
    Maps<S> M = raycast(X, P, Vol, load_pose<S>(T));
    for (uint8_t v : M.valid) hits += v;
  });
  return hits;
}

// Whole sequence: frame 0 at exp(seed) T0, then track/fuse/raycast per frame.
// depths: n_frames x H x W; depth_dots likewise or NULL.  poses_out:
// n_frames x 16 x ncomp.  stats_out (optional): n_frames x 6 doubles
// (lost, cnt of the last ICP pass, sum r^2 of that pass, fused voxels,
// raycast hits, sum of cnt over all ICP passes).  F_out/W_out (optional):
// final volume, x-fastest, ncomp per scalar.  sched_poses (n_frames x 16) and
// sched_params (mu, fx, fy, cx, cy), both optional, freeze the raycast march
// schedule (finite-difference pins only).
void orc_run_sequence(const OrcConfig* c, const OrcSeed* seed, int n_frames, const double* depths,
                      const double* depth_dots, const double* T0, double* poses_out, double* stats_out,
                      double* F_out, double* W_out, const double* sched_poses, const double* sched_params) {
  Ctx X{*c, *seed};
  ORC_DISPATCH(seed, {
    const int nc = NC<S>::n;
    Params<S> P = make_params<S>(X);
    State<S> St;
    state_init(X, St);
    St.T = seeded_initial_pose<S>(X, T0);
    St.Tprev = St.T;
    size_t n = size_t(c->width) * c->height;
    for (int k = 0; k < n_frames; ++k) {
      FrameStats fs;
      Sched sc;
      if (sched_poses) {
        for (int i = 0; i < 16; ++i) sc.T[i] = sched_poses[k * 16 + i];
        sc.mu = sched_params[0]; sc.fx = sched_params[1]; sc.fy = sched_params[2];
        sc.cx = sched_params[3]; sc.cy = sched_params[4];
      }
      frame_step(X, P, St, depths + k * n, depth_dots ? depth_dots + k * n : nullptr, fs,
                 sched_poses ? &sc : nullptr);
      store_pose(poses_out + k * 16 * nc, St.T);
      if (stats_out) {
        double* o = stats_out + k * 6;
        o[0] = fs.lost; o[1] = fs.cnt_last; o[2] = fs.r2_last; o[3] = double(fs.n_fused);
        o[4] = double(fs.n_hits); o[5] = double(fs.cnt_sum);
      }
    }
    if (F_out || W_out) vol_out(St.vol, F_out, W_out);
  });
}

// Numerics pins: f(x) = (e^x + x^3 + x)/(x + 1) (Sec. 3, the function of the
// AD/FD/CSFD comparison table) evaluated on a seeded scalar x + h i1 (+ h i2).
void orc_eval_f(const OrcSeed* seed, double x, double* out) {
  ORC_DISPATCH(seed, {
    S z = seeded<S>(x, seed->kind >= 1 ? seed->h : 0.0, seed->kind == 2 ? seed->h : 0.0);
    S f = (orc::exp(z) + z * z * z + z) / (z + S(1.0));
    put(out, f);
  });
}
// g(x, y) = sin(x y) e^y / (1 + x^2) + sqrt(x + y^2), x on i1 and y on i2
// (mixed second derivative for the symmetry pin of eq. csfd_hessian).
void orc_eval_g(const OrcSeed* seed, double x, double y, int x_on, int y_on, double* out) {
  ORC_DISPATCH(seed, {
    double h = seed->h;
    S zx = seeded<S>(x, (x_on & 1) ? h : 0.0, (x_on & 2) ? h : 0.0);
    S zy = seeded<S>(y, (y_on & 1) ? h : 0.0, (y_on & 2) ? h : 0.0);
    S g = orc::sin(zx * zy) * orc::exp(zy) / (S(1.0) + zx * zx) + orc::sqrt(zx + zy * zy);
    put(out, g);
  });
}

// Translational RMSE over the frames, without alignment: sqrt(mean |t_k - t_k^gt|^2).
// poses: n x 16 x ncomp; gt: n x 16 real.  out: ncomp doubles.
void orc_traj_err(const OrcSeed* seed, int n, const double* poses, const double* gt, double* out) {
  ORC_DISPATCH(seed, {
    const int nc = NC<S>::n;
    S acc(0.0);
    for (int k = 0; k < n; ++k)
      for (int r = 0; r < 3; ++r) {
        S d = get<S>(poses + (k * 16 + r * 4 + 3) * nc) - S(gt[k * 16 + r * 4 + 3]);
        acc = acc + d * d;
      }
    put(out, orc::sqrt(acc / S(double(n))));
  });
}

}  // extern "C"
