// Shared device-side types of the frame step: parameters, poses, SE(3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "jet.hpp"

namespace xs {

constexpr int kMaxDirs = 16;
constexpr int kBrick = 8;                 // TSDF bricks of 8^3 voxels, 512 contiguous voxels each
constexpr int kBrickVox = kBrick * kBrick * kBrick;
constexpr int kIcpThreads = 256;
constexpr int kMaxIcpBlocks = 1200;
constexpr int kCounters = 40;
constexpr double kTapBias = 1e-3;         // ICP tap choice floor(u + 1e-3), see k_icp

// Parameters of one context in kernel precision T (jets where perturbable).
template <typename T, int D, int Q>
struct KParams {
  using J = Jet<T, D, Q>;
  J fx, fy, cx, cy;        // level-0 intrinsics
  J mu, wcap;              // truncation distance, weight cap
  T dgate2;                // squared distance gate (real)
  T cos_agate;             // cosine of the angle gate (real)
  T disc_delta;            // discontinuity threshold (m)
  T bil_is, bil_ir;        // 1/(2 sigma_px^2), 1/(2 sigma_m^2)
  T pyr_gate;              // 3 sigma_m
  double bil_is_d, bil_ir_d, pyr_gate_d;   // the same in FP64 (FP32 runs measure real parts in FP64)
  T voxel;                 // voxel size s
  T half[3];               // L/2 per axis
  T near_m;
  int bil_radius;
  int W, H;                // level-0 image size
  int dim[3];              // voxels per axis (multiples of 8)
  int nbr[3];              // bricks per axis
  int wcap_dir;            // direction perturbing the weight cap, or -1
  int depth_plane[kMaxDirs];   // per direction: index of its depth_dot plane or -1
  T depth_h[kMaxDirs];         // per direction: step h (scales depth_dot)
};

// FP64 pose jets: R (row-major 3x3) then t; camera-to-world.
template <int D, int Q>
struct MPose {
  Jet<double, D, Q> m[12];
};
// the same in kernel precision
template <typename T, int D, int Q>
struct KPose {
  Jet<T, D, Q> R[9], t[3];
};

template <typename T, typename U, int D, int Q>
XJ KPose<T, D, Q> to_kpose(const MPose<D, Q>& P) {
  KPose<T, D, Q> k;
#pragma unroll
  for (int i = 0; i < 9; ++i) k.R[i] = jcast<T>(P.m[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) k.t[i] = jcast<T>(P.m[9 + i]);
  return k;
}

// R p + t, evaluated left to right
template <typename J, typename K>
XJ V3<J> pose_apply(const K& P, const V3<J>& p) {
  return {P.R[0] * p.x + P.R[1] * p.y + P.R[2] * p.z + P.t[0],
          P.R[3] * p.x + P.R[4] * p.y + P.R[5] * p.z + P.t[1],
          P.R[6] * p.x + P.R[7] * p.y + P.R[8] * p.z + P.t[2]};
}
template <typename J, typename K>
XJ V3<J> pose_rotate(const K& P, const V3<J>& p) {
  return {P.R[0] * p.x + P.R[1] * p.y + P.R[2] * p.z,
          P.R[3] * p.x + P.R[4] * p.y + P.R[5] * p.z,
          P.R[6] * p.x + P.R[7] * p.y + P.R[8] * p.z};
}
// R^T (p - t): transpose, never conjugate
template <typename J, typename K>
XJ V3<J> pose_apply_inv(const K& P, const V3<J>& p) {
  V3<J> d = {p.x - P.t[0], p.y - P.t[1], p.z - P.t[2]};
  return {P.R[0] * d.x + P.R[3] * d.y + P.R[6] * d.z,
          P.R[1] * d.x + P.R[4] * d.y + P.R[7] * d.z,
          P.R[2] * d.x + P.R[5] * d.y + P.R[8] * d.z};
}

// composition A * B of rigid transforms (FP64 jets)
template <int D, int Q>
XJ MPose<D, Q> pose_mul(const MPose<D, Q>& A, const MPose<D, Q>& B) {
  MPose<D, Q> C;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C.m[r * 3 + c] = A.m[r * 3 + 0] * B.m[0 * 3 + c] + A.m[r * 3 + 1] * B.m[1 * 3 + c] + A.m[r * 3 + 2] * B.m[2 * 3 + c];
    C.m[9 + r] = A.m[r * 3 + 0] * B.m[9 + 0] + A.m[r * 3 + 1] * B.m[9 + 1] + A.m[r * 3 + 2] * B.m[9 + 2] + A.m[9 + r];
  }
  return C;
}
template <int D, int Q>
XJ MPose<D, Q> pose_inverse(const MPose<D, Q>& A) {
  MPose<D, Q> I;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) I.m[r * 3 + c] = A.m[c * 3 + r];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    I.m[9 + r] = -(I.m[r * 3 + 0] * A.m[9] + I.m[r * 3 + 1] * A.m[10] + I.m[r * 3 + 2] * A.m[11]);
  return I;
}

// SE(3) exponential (Sec. 4.1 eqs. "lie", "rotvector", "rotation_jacobi"):
// theta^2 = phi.phi; R = I + A[phi]x + B[phi]x^2, V = I + B[phi]x + C[phi]x^2,
// t = V rho; A, B, C as even series in theta^2 below 1e-2 (the axis phi/theta is
// undefined at phi = 0 where every pose seed and ICP update starts), else
// sin/cos closed forms.
template <int D, int Q>
XJ void se3_abc(const Jet<double, D, Q> xi[6], Jet<double, D, Q>& A, Jet<double, D, Q>& B, Jet<double, D, Q>& C) {
  using J = Jet<double, D, Q>;
  const J& px = xi[0];
  const J& py = xi[1];
  const J& pz = xi[2];
  J t2 = px * px + py * py + pz * pz;
  if (t2.re() < 1e-2) {
    // (the coefficients 1/k! are rounded constants: a product per term
    // instead of a division, well inside the series' own truncation error)
    J t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4;
    A = jconst<J>(1.0) - t2 * (1.0 / 6.0) + t4 * (1.0 / 120.0) - t6 * (1.0 / 5040.0) + t8 * (1.0 / 362880.0);
    B = jconst<J>(0.5) - t2 * (1.0 / 24.0) + t4 * (1.0 / 720.0) - t6 * (1.0 / 40320.0) + t8 * (1.0 / 3628800.0);
    C = jconst<J>(1.0 / 6.0) - t2 * (1.0 / 120.0) + t4 * (1.0 / 5040.0) - t6 * (1.0 / 362880.0) +
        t8 * (1.0 / 39916800.0);
  } else {
    J th = jsqrt(t2);
    J s = jsin(th), c = jcos(th);
    A = s / th;
    B = (jconst<J>(1.0) - c) / t2;
    C = (th - s) / (t2 * th);
  }
}

template <int D, int Q>
XJ MPose<D, Q> se3_exp(const Jet<double, D, Q> xi[6]) {
  using J = Jet<double, D, Q>;
  const J& px = xi[0];
  const J& py = xi[1];
  const J& pz = xi[2];
  J A, B, C;
  se3_abc<D, Q>(xi, A, B, C);
  J z = jzero<J>();
  J K[9] = {z, -pz, py, pz, z, -px, -py, px, z};
  J K2[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) K2[r * 3 + c] = K[r * 3 + 0] * K[0 * 3 + c] + K[r * 3 + 1] * K[1 * 3 + c] + K[r * 3 + 2] * K[2 * 3 + c];
  MPose<D, Q> T;
  J Vm[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      J I = jconst<J>(r == c ? 1.0 : 0.0);
      T.m[r * 3 + c] = I + A * K[r * 3 + c] + B * K2[r * 3 + c];
      Vm[r * 3 + c] = I + B * K[r * 3 + c] + C * K2[r * 3 + c];
    }
#pragma unroll
  for (int r = 0; r < 3; ++r) T.m[9 + r] = Vm[r * 3 + 0] * xi[3] + Vm[r * 3 + 1] * xi[4] + Vm[r * 3 + 2] * xi[5];
  return T;
}

// One entry of exp(xi) * P, for one lane of a wave: row r (0..2) and column c
// (0..2 rotation, 3 translation) of the 3x4 result, with the arithmetic of
// se3_exp followed by pose_mul for that entry (each lane forms only row r of
// exp(xi); the rows of [phi]x it needs are picked with selects, not indexing).
template <int D, int Q>
__device__ __forceinline__ Jet<double, D, Q> se3_exp_mul_entry(const Jet<double, D, Q> xi[6],
                                                               const Jet<double, D, Q> col[3], int r, int c) {
  using J = Jet<double, D, Q>;
  const J& px = xi[0];
  const J& py = xi[1];
  const J& pz = xi[2];
  J A, B, C;
  se3_abc<D, Q>(xi, A, B, C);
  const J z = jzero<J>();
  const J K[9] = {z, -pz, py, pz, z, -px, -py, px, z};
  auto pick = [r](const J& a, const J& b, const J& d) { return r == 0 ? a : (r == 1 ? b : d); };
  const J Kr[3] = {pick(K[0], K[3], K[6]), pick(K[1], K[4], K[7]), pick(K[2], K[5], K[8])};
  J Er[3], Vr[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const J K2 = Kr[0] * K[0 * 3 + k] + Kr[1] * K[1 * 3 + k] + Kr[2] * K[2 * 3 + k];
    const J I = jconst<J>(r == k ? 1.0 : 0.0);
    Er[k] = I + A * Kr[k] + B * K2;
    Vr[k] = I + B * Kr[k] + C * K2;
  }
  const J tr = Vr[0] * xi[3] + Vr[1] * xi[4] + Vr[2] * xi[5];
  // column c of P: rotation column c, or the translation
  const J prod = Er[0] * col[0] + Er[1] * col[1] + Er[2] * col[2];
  return c < 3 ? prod : prod + tr;
}

// The same entries with the column read from P where it is used.
template <int D, int Q>
__device__ __forceinline__ Jet<double, D, Q> se3_exp_mul_entry(const Jet<double, D, Q> xi[6],
                                                               const MPose<D, Q>* __restrict__ P, int r, int c) {
  using J = Jet<double, D, Q>;
  const J& px = xi[0];
  const J& py = xi[1];
  const J& pz = xi[2];
  J A, B, C;
  se3_abc<D, Q>(xi, A, B, C);
  const J z = jzero<J>();
  const J K[9] = {z, -pz, py, pz, z, -px, -py, px, z};
  auto pick = [r](const J& a, const J& b, const J& d) { return r == 0 ? a : (r == 1 ? b : d); };
  const J Kr[3] = {pick(K[0], K[3], K[6]), pick(K[1], K[4], K[7]), pick(K[2], K[5], K[8])};
  J Er[3], Vr[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const J K2 = Kr[0] * K[0 * 3 + k] + Kr[1] * K[1 * 3 + k] + Kr[2] * K[2 * 3 + k];
    const J I = jconst<J>(r == k ? 1.0 : 0.0);
    Er[k] = I + A * Kr[k] + B * K2;
    Vr[k] = I + B * Kr[k] + C * K2;
  }
  const J tr = Vr[0] * xi[3] + Vr[1] * xi[4] + Vr[2] * xi[5];
  const J p0 = c < 3 ? P->m[0 * 3 + c] : P->m[9 + 0];
  const J p1 = c < 3 ? P->m[1 * 3 + c] : P->m[9 + 1];
  const J p2 = c < 3 ? P->m[2 * 3 + c] : P->m[9 + 2];
  const J prod = Er[0] * p0 + Er[1] * p1 + Er[2] * p2;
  return c < 3 ? prod : prod + tr;
}
template <int D, int Q>
__device__ __forceinline__ Jet<double, D, Q> smallangle_mul_entry(const Jet<double, D, Q> xi[6],
                                                                  const MPose<D, Q>* __restrict__ P, int r, int c) {
  using J = Jet<double, D, Q>;
  const J z = jzero<J>();
  const J K[9] = {z, -xi[2], xi[1], xi[2], z, -xi[0], -xi[1], xi[0], z};
  J Er[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) Er[k] = jconst<J>(r == k ? 1.0 : 0.0) + K[r * 3 + k];
  const J p0 = c < 3 ? P->m[0 * 3 + c] : P->m[9 + 0];
  const J p1 = c < 3 ? P->m[1 * 3 + c] : P->m[9 + 1];
  const J p2 = c < 3 ? P->m[2 * 3 + c] : P->m[9 + 2];
  const J prod = Er[0] * p0 + Er[1] * p1 + Er[2] * p2;
  return c < 3 ? prod : prod + xi[3 + r];
}

// Column c of the pose P (rotation column c < 3, else the translation), the
// operand of the *_mul_entry functions.
template <int D, int Q>
__device__ __forceinline__ void pose_column(const MPose<D, Q>* __restrict__ P, int c, Jet<double, D, Q> col[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) col[k] = c < 3 ? P->m[k * 3 + c] : P->m[9 + k];
}

// Entry (r, c) of T_sa(xi) * P with T_sa the small-angle transform of eq.
// icp_approx: rotation I + [phi]x (cos taken as 1, sin as the angle),
// translation rho.
template <int D, int Q>
__device__ __forceinline__ Jet<double, D, Q> smallangle_mul_entry(const Jet<double, D, Q> xi[6],
                                                                  const Jet<double, D, Q> col[3], int r, int c) {
  using J = Jet<double, D, Q>;
  const J z = jzero<J>();
  const J K[9] = {z, -xi[2], xi[1], xi[2], z, -xi[0], -xi[1], xi[0], z};
  J Er[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) Er[k] = jconst<J>(r == k ? 1.0 : 0.0) + K[r * 3 + k];
  const J prod = Er[0] * col[0] + Er[1] * col[1] + Er[2] * col[2];
  return c < 3 ? prod : prod + xi[3 + r];
}

// Two Newton steps of the polar decomposition, R <- 1.5 R - 0.5 R (R^T R),
// on a row-major 3x3 rotation estimate (quadratic convergence to the nearest
// rotation).
template <int D, int Q>
__device__ __forceinline__ void polar_steps(Jet<double, D, Q> R[9]) {
  using J = Jet<double, D, Q>;
  for (int it = 0; it < 2; ++it) {
    J G[9], N[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) G[a * 3 + b] = R[0 * 3 + a] * R[0 * 3 + b] + R[1 * 3 + a] * R[1 * 3 + b] + R[2 * 3 + a] * R[2 * 3 + b];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        N[a * 3 + b] = 1.5 * R[a * 3 + b] -
                       0.5 * (R[a * 3 + 0] * G[0 * 3 + b] + R[a * 3 + 1] * G[1 * 3 + b] + R[a * 3 + 2] * G[2 * 3 + b]);
#pragma unroll
    for (int q = 0; q < 9; ++q) R[q] = N[q];
  }
}

// brick layout: brick (bx,by,bz) of 8^3 voxels stored contiguously, x fastest inside
XJ int64_t vox_index(int i, int j, int k, const int nbr[3]) {
  int64_t b = (int64_t(k >> 3) * nbr[1] + (j >> 3)) * nbr[0] + (i >> 3);
  return b * kBrickVox + (((k & 7) * 8 + (j & 7)) * 8 + (i & 7));
}

}  // namespace xs
