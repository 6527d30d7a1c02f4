// Camera relocalisation objective (Sec. 5.2): the query depth fused into the
// reference volume at the candidate pose T_q gives F_q = surface_update(M_r,
// T_q, D_q), and E(T_q) = sum_p (F_r(p) - F_q(p))^2.  A voxel the update
// leaves alone contributes 0; an updated voxel has F_q = (W_r F_r + F_D) /
// (W_r + 1), so it contributes ((F_r - F_D) / (W_r + 1))^2.  Voxels the
// reference never observed (W_r = 0) carry no reference value and are left
// out.  Nothing is written to the volume.
//
// The update's decisions are fusion's, on real parts.  F_D is evaluated with
// the pose increment as six hyper-dual directions and their 21 pairs
// (Jet<T, 6, 6>) through the projection and the depth lookup's fractional
// weights, so one pass sums E with its gradient and Hessian in the left
// increment exp(delta) T_q: the six complex-step and 21 bicomplex runs of the
// surface update that the paper's optimiser takes per iteration, in one
// launch.  Real runs only: the increment's directions occupy the jet.
//
// Work: each workgroup takes bricks blockIdx.x + k gridDim.x in increasing k,
// tests 512 of them at a time (observed, and fusion's conservative cull for
// the query pose), compacts the survivors in index order in LDS, and runs one
// voxel per thread over them.  The partial sums are therefore deterministic;
// a fixed-order finish adds them.
#pragma once
#include "newton.hpp"

namespace xs {

constexpr int kRelocNS = 29;        // E, gradient 6, Hessian 21, count
constexpr int kRelocBlocks = 1024;  // fixed: the order of the FP64 sums

template <typename T>
__global__ __launch_bounds__(kBrickVox) void k_reloc(KParams<T, 0, 0> kp, const KPose<T, 0, 0>* __restrict__ Kq,
                                                     const T* __restrict__ Df, const T* __restrict__ tmax,
                                                     const T* __restrict__ cmax, const uint8_t* __restrict__ bflags,
                                                     const typename Vec2<T>::type* __restrict__ rec, int nbrick,
                                                     double* __restrict__ partials) {
  using JN = Jet<T, 6, 6>;
  using R0 = Jet<T, 0, 0>;
  constexpr int NS = kRelocNS;
  constexpr int NW = kBrickVox / 64;
  __shared__ double red[NW][NS];
  __shared__ int sl[kBrickVox];
  __shared__ int wc[NW], wb[NW], nsel;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int W = kp.W, H = kp.H;
  const KPose<T, 0, 0> P = *Kq;
  // The voxel centre seen from exp(delta) T_q is R_q^T (y - t_q) with
  // y = exp(delta)^-1 c = R_d^T (c - t_d); to second order in the hyper-dual
  // increment R_d^T = I - K + K^2 / 2 and t_d = rho + K rho / 2, K = [phi]x
  // (higher terms vanish in the jet).  phi, rho are unit jets, so y is cheap.
  V3<JN> phv, rhv;
  {
    JN* pc[3] = {&phv.x, &phv.y, &phv.z};
    JN* rc[3] = {&rhv.x, &rhv.y, &rhv.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      *pc[a] = jzero<JN>();
      pc[a]->v[1 + a] = T(1);
      *rc[a] = jzero<JN>();
      rc[a]->v[4 + a] = T(1);
    }
  }
  const V3<JN> kr = vcross(phv, rhv);
  const T R[9] = {P.R[0].re(), P.R[1].re(), P.R[2].re(), P.R[3].re(), P.R[4].re(),
                  P.R[5].re(), P.R[6].re(), P.R[7].re(), P.R[8].re()};
  const T tq[3] = {P.t[0].re(), P.t[1].re(), P.t[2].re()};
  const T fxr = kp.fx.re(), fyr = kp.fy.re(), cxr = kp.cx.re(), cyr = kp.cy.re(), mur = kp.mu.re();
  T acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0;
  for (int base = 0; int64_t(blockIdx.x) + int64_t(base) * gridDim.x < nbrick; base += kBrickVox) {
    // this workgroup's next 512 candidate bricks, the survivors compacted in order
    const int64_t bc = int64_t(blockIdx.x) + int64_t(base + t) * gridDim.x;
    const bool keep = bc < nbrick && (bflags[bc] & 1) && brick_may_update(kp, P, tmax, cmax, int(bc));
    const unsigned long long bal = __ballot(keep);
    if (lane == 0) wc[wv] = int(__popcll(bal));
    __syncthreads();
    if (t == 0) {
      int tot = 0;
      for (int w = 0; w < NW; ++w) {
        wb[w] = tot;
        tot += wc[w];
      }
      nsel = tot;
    }
    __syncthreads();
    if (keep) sl[wb[wv] + __popcll(bal & ((1ull << lane) - 1ull))] = int(bc);
    __syncthreads();
    const int ns = nsel;
    for (int q = 0; q < ns; ++q) {
      const int b = sl[q];
      const int bx = b % kp.nbr[0], by = (b / kp.nbr[0]) % kp.nbr[1], bz = b / (kp.nbr[0] * kp.nbr[1]);
      const int i = bx * 8 + (t & 7), j = by * 8 + ((t >> 3) & 7), k = bz * 8 + (t >> 6);
      const auto r = rec[int64_t(b) * kBrickVox + t];
      if (!(r.y > T(0))) continue;                       // unobserved in the reference
      T cc[3];
      voxel_centre(kp, i, j, k, cc);
      // ---- fusion's decisions, on real parts
      const V3<R0> cr = {jconst<R0>(cc[0]), jconst<R0>(cc[1]), jconst<R0>(cc[2])};
      const V3<R0> xr = pose_apply_inv(P, cr);
      if (!(xr.z.re() > T(0))) continue;
      const T ux_r = fxr * xr.x.re() / xr.z.re() + cxr;
      const T uy_r = fyr * xr.y.re() / xr.z.re() + cyr;
      const T fx0 = floor(ux_r), fy0 = floor(uy_r);
      if (!(fx0 >= T(0) && fy0 >= T(0) && fx0 <= T(W - 2) && fy0 <= T(H - 2))) continue;
      const int i0 = int(fx0), j0 = int(fy0);
      const size_t t0 = size_t(j0) * W + i0;
      const T d0 = Df[t0], d1 = Df[t0 + 1], d2 = Df[t0 + W], d3 = Df[t0 + W + 1];
      if (!(d0 > T(0) && d1 > T(0) && d2 > T(0) && d3 > T(0))) continue;
      const int in = int(floor(ux_r + T(0.5))), jn = int(floor(uy_r + T(0.5)));
      const T dn = Df[size_t(jn) * W + in];
      const T disc = fabs(d0 - dn) + fabs(d1 - dn) + fabs(d2 - dn) + fabs(d3 - dn);
      const bool nearest = disc >= kp.disc_delta;
      T Lr;
      if (nearest) {
        Lr = dn;
      } else {
        const T a = ux_r - fx0, bb = uy_r - fy0;
        const T a1 = T(1) - a, b1 = T(1) - bb;
        Lr = b1 * (a1 * d0 + a * d1) + bb * (a1 * d2 + a * d3);
      }
      if (Lr - xr.z.re() < -mur) continue;
      // ---- the contribution with its gradient and Hessian in the increment
      const V3<JN> w = {jconst<JN>(cc[0]) - rhv.x - T(0.5) * kr.x, jconst<JN>(cc[1]) - rhv.y - T(0.5) * kr.y,
                        jconst<JN>(cc[2]) - rhv.z - T(0.5) * kr.z};
      const V3<JN> kw = vcross(phv, w);
      const V3<JN> kkw = vcross(phv, kw);
      const JN y0 = w.x - kw.x + T(0.5) * kkw.x - tq[0];
      const JN y1 = w.y - kw.y + T(0.5) * kkw.y - tq[1];
      const JN y2 = w.z - kw.z + T(0.5) * kkw.z - tq[2];
      const V3<JN> x = {R[0] * y0 + R[3] * y1 + R[6] * y2, R[1] * y0 + R[4] * y1 + R[7] * y2,
                        R[2] * y0 + R[5] * y1 + R[8] * y2};
      JN L;
      if (nearest) {
        L = jconst<JN>(dn);                               // the nearest tap carries no coordinate tangent
      } else {
        const JN ux = fxr * x.x / x.z + cxr, uy = fyr * x.y / x.z + cyr;
        const JN a = ux - T(i0), bb = uy - T(j0);
        const JN a1 = jconst<JN>(T(1)) - a, b1 = jconst<JN>(T(1)) - bb;
        L = b1 * (a1 * d0 + a * d1) + bb * (a1 * d2 + a * d3);
      }
      const JN eta = L - x.z;
      const JN Fd = (eta.re() >= mur) ? jconst<JN>(T(1)) : eta / mur;
      const JN dlt = (jconst<JN>(r.x) - Fd) / (r.y + T(1));
      const JN e = dlt * dlt;
#pragma unroll
      for (int c2 = 0; c2 < 28; ++c2) acc[c2] += e.v[c2];
      acc[28] += T(1);
    }
    __syncthreads();   // sl, wc, wb and nsel are rewritten by the next round
  }
  {
    double tot[1];
    wave_sum_transposed<NS>(acc, lane, tot);
    if (lane < NS) red[wv][lane] = tot[0];
  }
  __syncthreads();
  double* part = partials + size_t(blockIdx.x) * NS;
  for (int k = t; k < NS; k += kBrickVox) {
    double s = red[0][k];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += red[w][k];
    part[k] = s;
  }
}

// Fixed-order cross-workgroup sums of k_reloc -> out[29]: 32 groups of
// workgroups (b = g + 32 m), each summed by one thread per column into 8
// running sums (m mod 8, all loads unrolled and in flight together), then a
// fixed pairwise tree over the groups.  (T: the context precision; one
// instance per shape.)
template <typename T>
__global__ __launch_bounds__(1024) void k_reloc_finish(const double* __restrict__ partials, double* __restrict__ out) {
  constexpr int NS = kRelocNS, G = 32, KC = 32, M = kRelocBlocks / G;
  static_assert(kRelocBlocks % (G * 8) == 0 && NS <= KC, "reloc finish shape");
  __shared__ double gs[G][KC];
  const int grp = threadIdx.x / KC, kk = threadIdx.x % KC;
  double a8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (kk < NS) {
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = partials[size_t(grp + m * G) * NS + kk];
#pragma unroll
    for (int m = 0; m < M; ++m) a8[m & 7] += v[m];
  }
  gs[grp][kk] = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
  __syncthreads();
  if (threadIdx.x < NS) {
    double s[G];
#pragma unroll
    for (int g = 0; g < G; ++g) s[g] = gs[g][threadIdx.x];
#pragma unroll
    for (int w = G / 2; w >= 1; w /= 2)
#pragma unroll
      for (int g = 0; g < w; ++g) s[g] = s[2 * g] + s[2 * g + 1];
    out[threadIdx.x] = s[0];
  }
}

}  // namespace xs
