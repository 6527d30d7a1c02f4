// Newton ICP (Sec. 4.1: a second-order ICP step with Newton's method, its
// Hessian by the multicomplex step of eq. csfd_hessian, no small-angle
// approximation).
//
// The objective of one pass is E(delta) = sum r(exp(delta) T_j)^2 over the
// correspondences.  Every pixel's residual is evaluated with the pose
// increment delta as six hyper-dual directions with all 21 pair parts
// (Jet<T, 6, 6>: the exact gradient and Hessian of r in delta at delta = 0).
// kHold (icp.solver 1) holds the pass's correspondences fixed: the looked-up
// model point and normal are constants of the pass, and the derivatives come
// from the pose's action on the measured point (its exponential map);
// otherwise (solver 2) they run through the whole association: projection,
// bilinear model lookup with its fractional weights (gates decided on real
// parts), so they include how the looked-up point and normal move.  The
// pass sums the 28 parts of r^2 (E, its gradient, its Hessian), and, for the
// fall-back step, the Gauss-Newton sums with the correspondences held fixed
// (A = sum J J^T, b = sum J r, J = [p x m; m]) and the count.  The finish
// solves (H/2) delta = -(g/2) when the Hessian's LDL^T pivots pass the
// solver's test, else the Gauss-Newton system, and updates the pose as the
// Gauss-Newton pass does.
//
// Real runs only (a perturbation with no directions): the increment's
// directions occupy the jet.
#pragma once
#include "kernels.hpp"

namespace xs {

// E (1), gradient (6), Hessian pairs (21), Gauss-Newton A (21) and b (6), count
constexpr int kNewtonNS = 28 + 21 + 6 + 1;
constexpr int kNewtonOut = 29;   // E, g[6], H[21] (upper triangle row-major), count

template <typename T, int D, int Q, bool kHold>
__global__ __launch_bounds__(kIcpThreads) void k_icp_newton(KParams<T, D, Q> kp, IcpArgs<T, D, Q> g) {
  using JN = Jet<T, 6, 6>;
  constexpr int NC = Jet<T, D, Q>::N;
  constexpr int NS = kNewtonNS;
  __shared__ double red[kIcpThreads / 64][NS];
  const KPose<T, D, Q> Kc = *g.Kcur;
  const KPose<T, D, Q> Kq = *g.Kprev;
  // exp(delta) T_j to second order in the hyper-dual increment:
  // R = I + K + K^2 / 2, t = rho + K rho / 2 with K = [phi]x (higher terms
  // are third order and vanish in the jet), composed with the real T_j
  JN ph[3], rh[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ph[a] = jzero<JN>();
    ph[a].v[1 + a] = T(1);
    rh[a] = jzero<JN>();
    rh[a].v[4 + a] = T(1);
  }
  const JN z = jzero<JN>();
  const JN K[9] = {z, -ph[2], ph[1], ph[2], z, -ph[0], -ph[1], ph[0], z};
  JN Ri[9], ti[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const JN K2 = K[r * 3 + 0] * K[0 * 3 + c] + K[r * 3 + 1] * K[1 * 3 + c] + K[r * 3 + 2] * K[2 * 3 + c];
      Ri[r * 3 + c] = jconst<JN>(T(r == c ? 1 : 0)) + K[r * 3 + c] + T(0.5) * K2;
    }
    ti[r] = rh[r] + T(0.5) * (K[r * 3 + 0] * rh[0] + K[r * 3 + 1] * rh[1] + K[r * 3 + 2] * rh[2]);
  }
  KPose<T, 6, 6> Tc, Tp;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Tc.R[r * 3 + c] = Ri[r * 3 + 0] * Kc.R[0 * 3 + c].re() + Ri[r * 3 + 1] * Kc.R[1 * 3 + c].re() +
                        Ri[r * 3 + 2] * Kc.R[2 * 3 + c].re();
      Tp.R[r * 3 + c] = jconst<JN>(Kq.R[r * 3 + c].re());
    }
    Tc.t[r] = Ri[r * 3 + 0] * Kc.t[0].re() + Ri[r * 3 + 1] * Kc.t[1].re() + Ri[r * 3 + 2] * Kc.t[2].re() + ti[r];
    Tp.t[r] = jconst<JN>(Kq.t[r].re());
  }
  const T sc = T(1) / T(1 << g.level);
  const JN fx = jconst<JN>(kp.fx.re() * sc), fy = jconst<JN>(kp.fy.re() * sc);
  const JN cx = jconst<JN>(kp.cx.re() * sc), cy = jconst<JN>(kp.cy.re() * sc);
  const size_t n = size_t(g.W) * g.H;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const size_t chunk = (n + size_t(gridDim.x) * kIcpThreads - 1) / (size_t(gridDim.x) * kIcpThreads) * kIcpThreads;
  const size_t p0 = size_t(xcd_remap(blockIdx.x, gridDim.x)) * chunk;
  const size_t p1 = p0 + chunk < n ? p0 + chunk : n;
  // maps hold real parts only here (component plane 0)
  auto ld = [&](const T* b, size_t idx) {
    V3<JN> v;
    JN* o[3] = {&v.x, &v.y, &v.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) *o[a] = jconst<JN>(b[size_t(a * NC) * n + idx]);
    return v;
  };
  T acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0;
  for (size_t i = p0 + threadIdx.x; i < p1; i += kIcpThreads) {
    JN jac[6], r;
    if (!icp_pixel_with<kHold>(kp, g, Tc, Tp, fx, fy, cx, cy, n, i, jac, r, ld)) continue;
    const JN rr = r * r;
#pragma unroll
    for (int c = 0; c < 28; ++c) acc[c] += rr.v[c];
    int k = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b, ++k) acc[28 + k] += jac[a].re() * jac[b].re();
#pragma unroll
    for (int a = 0; a < 6; ++a) acc[49 + a] += jac[a].re() * r.re();
    acc[55] += T(1);
  }
  {
    double tot[1];
    wave_sum_transposed<NS>(acc, lane, tot);
    if (lane < NS) red[wv][lane] = tot[0];
  }
  __syncthreads();
  double* part = g.partials + size_t(blockIdx.x) * NS;
  for (int k = threadIdx.x; k < NS; k += kIcpThreads) {
    double s = red[0][k];
#pragma unroll
    for (int w = 1; w < kIcpThreads / 64; ++w) s += red[w][k];
    part[k] = s;
  }
}

// Cross-workgroup sums of the Newton pass in a fixed order (16 interleaved
// groups of workgroups, 8 running sums each, then a fixed tree), then the
// Newton or Gauss-Newton step (or only the sums: E, g, H, count).
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_icp_newton_finish(IcpArgs<T, D, Q> g, int nblocks) {
  constexpr int NS = kNewtonNS;
  constexpr int NT = 256, G = 16, KC = 64, GPT = G * KC / NT;
  __shared__ double gs[G][KC];
  __shared__ double fin[NS];
  __shared__ double fnew[29], fgn[29];
  __shared__ double xs[1][6];
  const int lost = *g.lost;
  FinishPre<D, Q> pre;
  if (threadIdx.x < 64) pre = finish_preload(g, int(threadIdx.x));
  const int grp0 = threadIdx.x / KC, kk = threadIdx.x % KC;
  const unsigned B = nblocks;
  for (int kc = 0; kc < NS; kc += KC) {
    const int k = kc + kk;
#pragma unroll
    for (int gi = 0; gi < GPT; ++gi) {
      const int grp = grp0 + gi * (NT / KC);
      double a8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (k < NS) {
        unsigned m = 0;
        for (unsigned b = grp; b < B; b += G, ++m) a8[m & 7] += g.partials[size_t(b) * NS + k];
      }
      gs[grp][kk] = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
    }
    __syncthreads();
    if (threadIdx.x < KC && kc + int(threadIdx.x) < NS) {
      double s8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) s8[u] = gs[2 * u][threadIdx.x] + gs[2 * u + 1][threadIdx.x];
      fin[kc + threadIdx.x] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    }
    __syncthreads();
  }
  if (threadIdx.x >= 64 || lost) return;
  const int lane = threadIdx.x;
  if (!g.do_solve) {
    if (lane < 28) g.sums_out[lane] = fin[lane];
    if (lane == 28) g.sums_out[28] = fin[55];
    return;
  }
  // the two candidate systems in the layout of the Gauss-Newton finish
  // (A 21, b 6, count, sum r^2)
  if (lane < 21) {
    fnew[lane] = 0.5 * fin[7 + lane];
    fgn[lane] = fin[28 + lane];
  } else if (lane < 27) {
    fnew[lane] = 0.5 * fin[1 + (lane - 21)];
    fgn[lane] = fin[49 + (lane - 21)];
  } else if (lane == 27) {
    fnew[27] = fgn[27] = fin[55];
  } else if (lane == 28) {
    fnew[28] = fgn[28] = fin[0];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  Jet<double, 0, 0> probe[6];
  const bool newton = int(fnew[27]) >= 6 && icp_solve<0, 0>(fnew, probe, lane, xs);
  if (!newton && lane == 0) pre.crow[34] += 1;
  icp_finish_solve<T, D, Q>(g, newton ? fnew : fgn, lane, xs, pre);
}

}  // namespace xs
