// HIP kernels of the CSFD frame step (X-SLAM Sec. 4.1), templated over the
// kernel precision T (float: FP32-complex, double: FP64-complex), the number of
// directions D and the Hessian size Q.  Decisions (validity, floors, gates,
// crossings, update masks) are taken on real parts evaluated with the same
// operations as a real run; the imaginary parts ride along.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>
#include "common.hpp"

namespace xs {

template <typename T> struct Vec2;
template <> struct Vec2<float> { typedef float2 type; };
template <> struct Vec2<double> { typedef double2 type; };

// Workgroups are dispatched to the 8 XCDs (each with its own L2) round-robin
// by linear workgroup id.  xcd_remap turns the physical id into a logical one
// such that every XCD receives a contiguous range of logical ids, so that
// neighbouring pixels (and the map rows or voxels they share) meet in the same
// L2.  A bijection of [0, n).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_remap(int id, int n) {
  const int x = id % kXcds, k = id / kXcds, q = n / kXcds, r = n % kXcds;
  return x * q + min(x, r) + k;
}

// The workgroup a kernel body works on: its position in the body's own grid
// and that grid's size.  A plain launch passes the hardware ids; a grouped
// launch (group.hpp) runs the bodies of several instances in one grid and
// passes each workgroup's position in its instance's grid.
// Pointers a body takes from a descriptor in memory: PtrSame leaves them as
// they are (kernel arguments, known to be global); PtrGlobal states that they
// address global memory, so that the accesses through them are global rather
// than flat instructions.
struct PtrSame {
  template <class P> __device__ __forceinline__ P* operator()(P* p) const { return p; }
};
struct PtrGlobal {
  template <class P> __device__ __forceinline__ P* operator()(P* p) const {
    return (P*)(P __attribute__((address_space(1)))*)(uintptr_t)p;
  }
};

struct VB {
  int bx, by, gx, gy;
  static __device__ __forceinline__ VB hw() {
    return VB{int(blockIdx.x), int(blockIdx.y), int(gridDim.x), int(gridDim.y)};
  }
};

// ---------------------------------------------------------------------------
// A1. depth promotion (eq. "csfd_depth") and bilateral filter
// ---------------------------------------------------------------------------
// Bilateral filter (Sec. 4.1 "Surface measurement"): normalised weighted sum
// over the valid pixels of a (2r+1)^2 window with weights
// exp(-|u-u'|^2/(2 s_px^2) - (D(u)-D(u'))^2/(2 s_m^2)), complex through D.
// The raw depth of a 16x16 tile plus its halo is staged in LDS (real parts and
// the depth tangents), one thread per output pixel.
constexpr int kBilTile = 16;
constexpr int kBilMaxR = 4;
template <typename T, int D, int Q> struct TrackBegin;
template <typename T, int D, int Q> __device__ void track_begin_work(const TrackBegin<T, D, Q>& a);
// (tb.lost != nullptr: workgroup 0 also starts the tracking of the frame,
// which only the kernels after this one read; see k_track_begin)
template <typename T, int D, int Q>
__device__ __forceinline__ void bilateral_body(const VB& vb, const KParams<T, D, Q>& kp, const T* __restrict__ depth,
                                                             const T* __restrict__ ddot, T* __restrict__ Dout,
                                                             double* __restrict__ Dhi, const TrackBegin<T, D, Q>& tb) {
  if (tb.lost && vb.bx == 0 && vb.by == 0 && threadIdx.x == 0 && threadIdx.y == 0) track_begin_work(tb);
  // FP32 runs evaluate the real part in FP64 as well (Dhi) and store it rounded:
  // normals are differences of neighbouring vertices a few mm apart at metres of
  // depth, which FP32 accumulation would leave with ~1e-4 rad errors
  constexpr bool kHi = std::is_same<T, float>::value;
  using J = Jet<T, D, Q>;
  constexpr int S = kBilTile + 2 * kBilMaxR;
  __shared__ J tile[S * S];
  const int W = kp.W, H = kp.H, r = kp.bil_radius;
  const size_t n = size_t(W) * H;
  const int x0 = vb.bx * kBilTile - kBilMaxR, y0 = vb.by * kBilTile - kBilMaxR;
  const int tid = threadIdx.y * kBilTile + threadIdx.x;
  // the tile's raw depths and depth tangents, every load in flight together
  // (coordinates clamped to the image; entries outside it are zero), then
  // promoted to jets: D + h_d ddot_d e_d for a finite positive depth (eq.
  // "csfd_depth"; only the depth directions carry a tangent), else 0
  constexpr int NQ = (S * S + kBilTile * kBilTile - 1) / (kBilTile * kBilTile);
  T dv[NQ], tv[NQ][D > 0 ? D : 1];
  bool in[NQ];
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int q = tid + u * kBilTile * kBilTile;
    const int xx = x0 + q % S, yy = y0 + q / S;
    in[u] = q < S * S && xx >= 0 && yy >= 0 && xx < W && yy < H;
    const size_t qi = size_t(yy < 0 ? 0 : (yy >= H ? H - 1 : yy)) * W + (xx < 0 ? 0 : (xx >= W ? W - 1 : xx));
    dv[u] = depth[qi];
#pragma unroll
    for (int k = 0; k < D; ++k) tv[u][k] = kp.depth_plane[k] >= 0 ? ddot[size_t(kp.depth_plane[k]) * n + qi] : T(0);
  }
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    pin(dv[u]);
#pragma unroll
    for (int k = 0; k < D; ++k) pin(tv[u][k]);
  }
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int q = tid + u * kBilTile * kBilTile;
    if (q >= S * S) continue;
    J v = jzero<J>();
    if (in[u] && dv[u] > T(0) && isfinite(dv[u])) {
      v.v[0] = dv[u];
#pragma unroll
      for (int k = 0; k < D; ++k)
        if (kp.depth_plane[k] >= 0) v.v[1 + k] = kp.depth_h[k] * tv[u][k];
    }
    tile[q] = v;
  }
  __syncthreads();
  const int x = vb.bx * kBilTile + threadIdx.x, y = vb.by * kBilTile + threadIdx.y;
  if (x >= W || y >= H) return;
  const size_t i = size_t(y) * W + x;
  const J c = tile[(threadIdx.y + kBilMaxR) * S + threadIdx.x + kBilMaxR];
  if (!(c.re() > T(0)) || r <= 0) {
    jstore(Dout, n, i, c);
    if constexpr (kHi) Dhi[i] = double(c.re());
    return;
  }
  J num = jzero<J>(), den = jzero<J>();
  double num_hi = 0.0, den_hi = 0.0;
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx) {
      int xx = x + dx, yy = y + dy;
      if (xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
      const J d = tile[(threadIdx.y + kBilMaxR + dy) * S + threadIdx.x + kBilMaxR + dx];
      if (!(d.re() > T(0))) continue;
      J dd = c - d;
      J arg = jconst<J>(T(dx * dx + dy * dy) * kp.bil_is) + (dd * dd) * kp.bil_ir;
      J w;
      if constexpr (kHi) {
        // one exponential per tap, in FP64; the jet weight takes it rounded
        // as its value and for the chain rule of its imaginary parts
        const double ddh = double(c.re()) - double(d.re());
        const double wh = exp(-(double(dx * dx + dy * dy) * kp.bil_is_d + (ddh * ddh) * kp.bil_ir_d));
        num_hi = num_hi + wh * double(d.re());
        den_hi = den_hi + wh;
        const T e = T(wh);
        w = chain(-arg, e, e, e);
      } else {
        w = jexp(-arg);
      }
      num = num + w * d;
      den = den + w;
    }
  J out = num / den;
  if constexpr (kHi) {
    const double oh = num_hi / den_hi;
    Dhi[i] = oh;
    out.v[0] = float(oh);
  }
  jstore(Dout, n, i, out);
}
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_bilateral(KParams<T, D, Q> kp, const T* __restrict__ depth,
                                                   const T* __restrict__ ddot, T* __restrict__ Dout,
                                                   double* __restrict__ Dhi, TrackBegin<T, D, Q> tb) {
  bilateral_body<T, D, Q>(VB::hw(), kp, depth, ddot, Dout, Dhi, tb);
}

// Coarser level (Sec. 4.1: "Gaussian smoothing", the perturbation smoothed
// alike): 5x5 binomial (1,4,6,4,1)^2 centred on (2x,2y) over valid taps within
// 3 s_m of the centre, renormalised; real weights.
template <typename T, int D, int Q>
__device__ __forceinline__ void pyrdown_body(const VB& vb, const KParams<T, D, Q>& kp, const T* __restrict__ Din, int Wi, int Hi,
                                                           T* __restrict__ Dout, const double* __restrict__ Dhi_in,
                                                           double* __restrict__ Dhi_out) {
  using J = Jet<T, D, Q>;
  constexpr bool kHi = std::is_same<T, float>::value;   // FP32 runs: real part in FP64 as well
  const int Wo = Wi / 2, Ho = Hi / 2;
  const int x = vb.bx * 16 + threadIdx.x, y = vb.by * 16 + threadIdx.y;
  if (x >= Wo || y >= Ho) return;
  const size_t ni = size_t(Wi) * Hi, no = size_t(Wo) * Ho, o = size_t(y) * Wo + x;
  // the real parts of the 25 taps, all in flight together (indexes clamped
  // to the image; taps outside it are dropped); the centre is tap 12
  T dr[25];
  double dh[25];
  uint32_t qi[25];   // (an image holds far fewer than 2^32 pixels)
  bool inb[25];
#pragma unroll
  for (int t = 0; t < 25; ++t) {
    const int xx = 2 * x + t % 5 - 2, yy = 2 * y + t / 5 - 2;
    inb[t] = xx >= 0 && yy >= 0 && xx < Wi && yy < Hi;
    qi[t] = uint32_t(yy < 0 ? 0 : (yy >= Hi ? Hi - 1 : yy)) * uint32_t(Wi) + uint32_t(xx < 0 ? 0 : (xx >= Wi ? Wi - 1 : xx));
    dr[t] = Din[qi[t]];
    dh[t] = 0.0;
    if constexpr (kHi) dh[t] = Dhi_in[qi[t]];
  }
#pragma unroll
  for (int t = 0; t < 25; ++t) {
    pin(dr[t]);
    if constexpr (kHi) pin(dh[t]);
  }
  const T c = dr[12];
  if (!(c > T(0))) {
    jstore(Dout, no, o, jzero<J>());
    if constexpr (kHi) Dhi_out[o] = 0.0;
    return;
  }
  const int g[5] = {1, 4, 6, 4, 1};
  J num = jzero<J>();
  T den = 0;
  double num_hi = 0.0, den_hi = 0.0;
  const double ch = dh[12];
#pragma unroll
  for (int t = 0; t < 25; ++t) {
    bool ok = inb[t] && dr[t] > T(0);
    if constexpr (kHi) ok = ok && !(fabs(dh[t] - ch) > kp.pyr_gate_d);
    else ok = ok && !(fabs(dr[t] - c) > kp.pyr_gate);
    J tap;
    tap.v[0] = dr[t];
#pragma unroll
    for (int q = 1; q < J::N; ++q) tap.v[q] = Din[size_t(q) * ni + qi[t]];
    const int wi = g[t % 5] * g[t / 5];
    const T w = T(wi);
    const J numw = num + w * tap;
    num = ok ? numw : num;
    den = ok ? den + w : den;
    if constexpr (kHi) {
      const double wh = double(wi);
      num_hi = ok ? num_hi + wh * dh[t] : num_hi;
      den_hi = ok ? den_hi + wh : den_hi;
    }
  }
  J out = num / den;
  if constexpr (kHi) {
    const double oh = num_hi / den_hi;
    Dhi_out[o] = oh;
    out.v[0] = float(oh);
  }
  jstore(Dout, no, o, out);
}
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_pyrdown(KParams<T, D, Q> kp, const T* __restrict__ Din, int Wi, int Hi,
                                                 T* __restrict__ Dout, const double* __restrict__ Dhi_in,
                                                 double* __restrict__ Dhi_out) {
  pyrdown_body<T, D, Q>(VB::hw(), kp, Din, Wi, Hi, Dout, Dhi_in, Dhi_out);
}

// ---------------------------------------------------------------------------
// A2. vertex and normal maps (eqs. "vertex", "normal"), level l with K / 2^l.
// N = normalize((V(u_y+) - V(u)) x (V(u_x+) - V(u))) faces the camera.
// ---------------------------------------------------------------------------
// The three levels in one launch: a 1-D grid of 16x16 tiles, level 0's
// first, then level 1's and level 2's.
template <typename T>
struct VNLevels {
  const T* D[3];
  const double* Dhi[3];
  T* V[3];
  T* N[3];
  uint8_t* valid[3];
  int W[3], H[3];
  int tiles_x[3], first[4];   // tiles per row; first tile of each level (first[3] = total)
};
template <typename T, int D, int Q>
__device__ __forceinline__ void vertex_normal_px(const KParams<T, D, Q>& kp, int level, const T* __restrict__ Dl,
                                                 int Wl, int Hl, T* __restrict__ Vout, T* __restrict__ Nout,
                                                 uint8_t* __restrict__ valid, const double* __restrict__ Dhi,
                                                 int x, int y);
template <typename T, int D, int Q, class PtrAs = PtrSame>
__device__ __forceinline__ void vertex_normal_body(const VB& vb, const KParams<T, D, Q>& kp, const VNLevels<T>& lv,
                                                   const PtrAs& as = PtrAs()) {
  const int b = vb.bx;
  const int l = b < lv.first[1] ? 0 : (b < lv.first[2] ? 1 : 2);
  const int t = b - lv.first[l];
  const int x = (t % lv.tiles_x[l]) * 16 + threadIdx.x, y = (t / lv.tiles_x[l]) * 16 + threadIdx.y;
  vertex_normal_px(kp, l, as(lv.D[l]), lv.W[l], lv.H[l], as(lv.V[l]), as(lv.N[l]), as(lv.valid[l]), as(lv.Dhi[l]), x,
                   y);
}
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_vertex_normal(KParams<T, D, Q> kp, VNLevels<T> lv) {
  vertex_normal_body<T, D, Q>(VB::hw(), kp, lv);
}
template <typename T, int D, int Q>
__device__ __forceinline__ void vertex_normal_px(const KParams<T, D, Q>& kp, int level, const T* __restrict__ Dl,
                                                 int Wl, int Hl, T* __restrict__ Vout, T* __restrict__ Nout,
                                                 uint8_t* __restrict__ valid, const double* __restrict__ Dhi,
                                                 int x, int y) {
  // FP32 runs: the real parts of vertices and normals from the FP64 depth
  constexpr bool kHi = std::is_same<T, float>::value;
  using J = Jet<T, D, Q>;
  if (x >= Wl || y >= Hl) return;
  const size_t n = size_t(Wl) * Hl, i = size_t(y) * Wl + x;
  const T sc = T(1) / T(1 << level);
  const J fx = kp.fx * sc, fy = kp.fy * sc, cx = kp.cx * sc, cy = kp.cy * sc;
  // the depth (and FP64 real depth) of the pixel and of its right and lower
  // neighbours, loaded together (a neighbour outside the image is replaced by
  // the pixel itself and not used)
  const size_t i1 = x + 1 < Wl ? i + 1 : i, i2 = y + 1 < Hl ? i + Wl : i;
  J dj[3] = {jload<J>(Dl, n, i), jload<J>(Dl, n, i1), jload<J>(Dl, n, i2)};
  double dhi[3] = {0.0, 0.0, 0.0};
  if constexpr (kHi) {
    dhi[0] = Dhi[i];
    dhi[1] = Dhi[i1];
    dhi[2] = Dhi[i2];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pin(dj[k]);
    pin(dhi[k]);
  }
  auto vert = [&](int xx, int yy, const J& d, bool& ok) -> V3<J> {
    ok = d.re() > T(0);
    J rx = (jconst<J>(T(xx)) - cx) / fx;
    J ry = (jconst<J>(T(yy)) - cy) / fy;
    return {d * rx, d * ry, d};
  };
  // FP64 real vertex (FP32 runs)
  const double fxh = double(kp.fx.re()) * double(sc), fyh = double(kp.fy.re()) * double(sc);
  const double cxh = double(kp.cx.re()) * double(sc), cyh = double(kp.cy.re()) * double(sc);
  auto vert_hi = [&](int xx, int yy, double d, double v[3]) {
    v[0] = d * ((double(xx) - cxh) / fxh);
    v[1] = d * ((double(yy) - cyh) / fyh);
    v[2] = d;
  };
  bool ok0;
  V3<J> v0 = vert(x, y, dj[0], ok0);
  const J z = jzero<J>();
  double h0[3] = {0, 0, 0};
  if constexpr (kHi) {
    vert_hi(x, y, dhi[0], h0);
    if (ok0) { v0.x.v[0] = float(h0[0]); v0.y.v[0] = float(h0[1]); v0.z.v[0] = float(h0[2]); }
  }
  vstore(Vout, n, i, ok0 ? v0 : V3<J>{z, z, z});
  bool okn = false;
  V3<J> nn = {z, z, z};
  if (ok0 && x + 1 < Wl && y + 1 < Hl) {
    bool ok1, ok2;
    V3<J> v1 = vert(x + 1, y, dj[1], ok1);
    V3<J> v2 = vert(x, y + 1, dj[2], ok2);
    if (ok1 && ok2) {
      V3<J> a = vsub(v1, v0), b = vsub(v2, v0);
      V3<J> c = vcross(b, a);
      J cc = vdot(c, c);
      if constexpr (kHi) {
        double h1[3], h2[3];
        vert_hi(x + 1, y, dhi[1], h1);
        vert_hi(x, y + 1, dhi[2], h2);
        const double ah[3] = {h1[0] - h0[0], h1[1] - h0[1], h1[2] - h0[2]};
        const double bh[3] = {h2[0] - h0[0], h2[1] - h0[1], h2[2] - h0[2]};
        const double ch[3] = {bh[1] * ah[2] - bh[2] * ah[1], bh[2] * ah[0] - bh[0] * ah[2], bh[0] * ah[1] - bh[1] * ah[0]};
        const double cch = ch[0] * ch[0] + ch[1] * ch[1] + ch[2] * ch[2];
        if (cch > 0.0) {
          J inv = jconst<J>(T(1)) / jsqrt(cc);
          nn = vscale(inv, c);
          const double ih = 1.0 / sqrt(cch);
          nn.x.v[0] = float(ch[0] * ih);
          nn.y.v[0] = float(ch[1] * ih);
          nn.z.v[0] = float(ch[2] * ih);
          okn = true;
        }
      } else if (cc.re() > T(0)) {
        J inv = jconst<J>(T(1)) / jsqrt(cc);
        nn = vscale(inv, c);
        okn = true;
      }
    }
  }
  vstore(Nout, n, i, nn);
  valid[i] = okn ? 1 : 0;
}

// ---------------------------------------------------------------------------
// A3-A5. projective association, point-to-plane residual and Jacobian, the
// 6x6 normal equations, and (last block) the FP64 solve and SE(3) update.
// ---------------------------------------------------------------------------
template <typename T, int D, int Q>
struct IcpArgs {
  const T* V; const T* N; const uint8_t* valid;               // current level (camera frame)
  const T* Vm; const T* Nm; const T* Zm; const uint8_t* validm;  // model level (world frame)
  int W, H, level, iter_slot, do_solve;
  int update;                  // 0 exact exponential, 1 small-angle matrix + polar steps
  KPose<T, D, Q>* Kcur;        // current estimate (kernel precision), updated by the last block
  const KPose<T, D, Q>* Kprev; // projection reference T_{k-1}
  MPose<D, Q>* Pcur;           // current estimate (FP64 master)
  Jet<double, D, Q> omega;     // step relaxation of this level
  double* partials;            // [blocks][NS]
  int* lost;
  int32_t* counters;           // counter rows (base)
  const int* frame;            // device frame index
  int max_frames;
  double* sums_out;            // icp_pass: [NS] FP64 sums
};

template <int D, int Q> struct IcpSize {
  static constexpr int NC = Jet<float, D, Q>::N;
  static constexpr int NS = 27 * NC + 2;
};

// per-frame counter row: 0 lost, 1 fused voxels, 2 raycast hits, 3 sum of ICP
// correspondences, 4 last-pass correspondences, 5..29 per-pass correspondences,
// 30 active bricks, 31 raycast samples, 32 first pass (1-based) whose update
// norm fell below 1e-6 (0: never), 33 initialiser used (0 previous / constant
// velocity, 1 network)
constexpr int kMaxPasses = 25;
__device__ __forceinline__ int32_t* counter_row(int32_t* base, const int* frame, int max_frames) {
  return base + kCounters * min(*frame, max_frames - 1);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The wave sums of NS per-lane values, each bit for bit what wave_sum gives
// (the same butterfly: at every step a lane adds its partner's value to its
// own), but exchanging only the half of the values that is still needed: at
// the step of lane bit o a lane keeps one half of its current range and sends
// the other.  63 M double exchanges instead of 6 NS (M = ceil(NS / 64)); lane
// l ends with the totals of values l M .. l M + M - 1 (zero past NS).
template <int NS, typename A>
__device__ __forceinline__ void wave_sum_transposed(const A (&acc)[NS], int lane, double (&out)[(NS + 63) / 64]) {
  constexpr int M = (NS + 63) / 64, V = 64 * M;
  double a[V / 2];
  {
    const bool up = (lane & 32) != 0;
#pragma unroll
    for (int i = 0; i < V / 2; ++i) {
      const double lo = i < NS ? double(acc[i]) : 0.0;
      const double hi = i + V / 2 < NS ? double(acc[i + V / 2]) : 0.0;
      const double keep = up ? hi : lo, send = up ? lo : hi;
      a[i] = keep + __shfl_xor(send, 32, 64);
    }
  }
#pragma unroll
  for (int o = 16, L = V / 2; o >= 1; o >>= 1, L >>= 1) {
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < L / 2; ++i) {
      const double keep = up ? a[i + L / 2] : a[i], send = up ? a[i] : a[i + L / 2];
      a[i] = keep + __shfl_xor(send, o, 64);
    }
  }
#pragma unroll
  for (int j = 0; j < M; ++j) out[j] = a[j];
}

// Component C of the jet product x * y, by the same operations as the jet
// operator (so the same bits): real part, first-order part, or the part of
// the pair (a, b) of the first Q directions (row-major upper triangle).
template <int Q>
__host__ __device__ constexpr int pair_a(int p) {
  int a = 0;
  while (p >= Q - a) { p -= Q - a; ++a; }
  return a;
}
template <int Q>
__host__ __device__ constexpr int pair_b(int p) {
  int a = 0;
  while (p >= Q - a) { p -= Q - a; ++a; }
  return a + p;
}
template <int C, typename T, int D, int Q>
__device__ __forceinline__ T jet_prod_comp(const Jet<T, D, Q>& x, const Jet<T, D, Q>& y) {
  if constexpr (C == 0) {
    return x.v[0] * y.v[0];
  } else if constexpr (C <= D) {
    return tfma(x.v[0], y.v[C], x.v[C] * y.v[0]);
  } else {
    constexpr int a = pair_a<Q>(C - 1 - D), b = pair_b<Q>(C - 1 - D);
    T s = tfma(x.v[0], y.v[C], x.v[C] * y.v[0]);
    s = tfma(x.v[1 + a], y.v[1 + b], s);
    return tfma(x.v[1 + b], y.v[1 + a], s);
  }
}
// Flat index F over the 27 normal-equation products (21 J_a J_b with a <= b,
// then 6 J_a r) and their non-real components 1..NC-1 (product-major).
__host__ __device__ constexpr int jj_a(int k) {
  int a = 0;
  while (k >= 6 - a) { k -= 6 - a; ++a; }
  return a;
}
__host__ __device__ constexpr int jj_b(int k) {
  int a = 0;
  while (k >= 6 - a) { k -= 6 - a; ++a; }
  return a + k;
}
template <int F, typename T, int D, int Q>
__device__ __forceinline__ double icp_flat_comp(const Jet<T, D, Q> (&jac)[6], const Jet<T, D, Q>& r) {
  constexpr int NT = Jet<T, D, Q>::N - 1;
  if constexpr (F >= 27 * NT) {
    return 0.0;
  } else {
    constexpr int k = F / NT, c = 1 + F % NT;
    if constexpr (k < 21)
      return double(jet_prod_comp<c>(jac[jj_a(k)], jac[jj_b(k)]));
    else
      return double(jet_prod_comp<c>(jac[k - 21], r));
  }
}
template <int F0, typename T, int D, int Q, int... J>
__device__ __forceinline__ void icp_fill_chunk(const Jet<T, D, Q> (&jac)[6], const Jet<T, D, Q>& r,
                                               double (&vals)[64], std::integer_sequence<int, J...>) {
  ((vals[J] = icp_flat_comp<F0 + J>(jac, r)), ...);
}
// Wave sums of every non-real component of one pixel's 27 products, 64 at a
// time with the half-exchanging butterfly (each sum bit for bit a wave_sum),
// added into the wave's row of LDS sums.  The row has NCO parts per product
// and part c of the jet goes to part PM::at(c) (a chunk of a wider jet).
struct SameParts {
  __host__ __device__ static constexpr int at(int c) { return c; }
};
template <typename T, int D, int Q, int NCO = Jet<T, D, Q>::N, typename PM = SameParts, int... CH>
__device__ __forceinline__ void icp_tangent_sums(const Jet<T, D, Q> (&jac)[6], const Jet<T, D, Q>& r, int lane,
                                                 double* red_row, std::integer_sequence<int, CH...>) {
  constexpr int NC = Jet<T, D, Q>::N, NT = NC - 1;
  auto one = [&](auto chi) {
    constexpr int ch = decltype(chi)::value;
    double vals[64];
    icp_fill_chunk<ch * 64>(jac, r, vals, std::make_integer_sequence<int, 64>{});
    double tot[1];
    wave_sum_transposed<64>(vals, lane, tot);
    const int f = ch * 64 + lane;
    if (f < 27 * NT) red_row[(f / NT) * NCO + PM::at(1 + f % NT)] += tot[0];
  };
  (one(std::integral_constant<int, CH>{}), ...);
}

// 6x6 symmetric solve with a real LDL^T factorisation of the real part and
// first/second-order parts from A x = -b differentiated (no conjugation).
// Called by the 64 lanes of one wave with the same sums: every lane factors
// and solves the real part; with several imaginary parts, direction d is
// solved on lane d - 1 and pair p on lane p (their right-hand sides need the
// directions' solutions, exchanged through Xs in LDS), each part with the
// operations of the serial order.
template <int D, int Q>
__device__ bool icp_solve(const double* sums, Jet<double, D, Q> dx[6], int lane, double (*Xs)[6]) {
  constexpr int NC = Jet<double, D, Q>::N;
  double A0[6][6], L[6][6], dd[6];
  int k = 0;
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b, ++k) { A0[a][b] = sums[k * NC]; A0[b][a] = sums[k * NC]; }
  double dmax = 0.0;
  for (int a = 0; a < 6; ++a) dmax = fmax(dmax, A0[a][a]);
  // (one division per pivot: the factor and the solves multiply by 1/d_j)
  double idd[6];
  for (int j = 0; j < 6; ++j) {
    double s = A0[j][j];
    for (int q = 0; q < j; ++q) s -= L[j][q] * L[j][q] * dd[q];
    if (!(s > 1e-12 * dmax)) return false;
    dd[j] = s;
    idd[j] = 1.0 / s;
    L[j][j] = 1.0;
    for (int i = j + 1; i < 6; ++i) {
      double t = A0[i][j];
      for (int q = 0; q < j; ++q) t -= L[i][q] * L[j][q] * dd[q];
      L[i][j] = t * idd[j];
    }
  }
  auto solve = [&](const double rhs[6], double x[6]) {
    double y[6];
    for (int i = 0; i < 6; ++i) {
      double t = rhs[i];
      for (int q = 0; q < i; ++q) t -= L[i][q] * y[q];
      y[i] = t;
    }
    for (int i = 5; i >= 0; --i) {
      double t = y[i] * idd[i];
      for (int q = i + 1; q < 6; ++q) t -= L[q][i] * x[q];
      x[i] = t;
    }
  };
  // component c of the symmetric matrix / vector
  auto Amul = [&](int c, const double v[6], double out[6]) {
    for (int a = 0; a < 6; ++a) out[a] = 0.0;
    int kk = 0;
    for (int a = 0; a < 6; ++a)
      for (int b = a; b < 6; ++b, ++kk) {
        double m = sums[kk * NC + c];
        out[a] += m * v[b];
        if (b != a) out[b] += m * v[a];
      }
  };
  double rhs[6], t1[6], t2[6];
  if constexpr (NC <= 2) {
    double X[NC][6];
    for (int a = 0; a < 6; ++a) rhs[a] = -sums[(21 + a) * NC];
    solve(rhs, X[0]);
    for (int d = 1; d <= D; ++d) {
      Amul(d, X[0], t1);
      for (int a = 0; a < 6; ++a) rhs[a] = -(sums[(21 + a) * NC + d] + t1[a]);
      solve(rhs, X[d]);
    }
    for (int a = 0; a < 6; ++a)
      for (int c = 0; c < NC; ++c) dx[a].v[c] = X[c][a];
  } else {
    static_assert(D <= 64 && Q * (Q + 1) / 2 <= 64, "one lane per imaginary part");
    constexpr int P = Q * (Q + 1) / 2;
    double X0[6], x[6];
    for (int a = 0; a < 6; ++a) rhs[a] = -sums[(21 + a) * NC];
    solve(rhs, X0);
    if (lane == 0)
      for (int a = 0; a < 6; ++a) Xs[0][a] = X0[a];
    if (lane < D) {
      const int d = lane + 1;
      Amul(d, X0, t1);
      for (int a = 0; a < 6; ++a) rhs[a] = -(sums[(21 + a) * NC + d] + t1[a]);
      solve(rhs, x);
      for (int a = 0; a < 6; ++a) Xs[d][a] = x[a];
    }
    // (one wave: its LDS accesses complete in program order)
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
    if (lane < P) {
      const int a = pair_a<Q>(lane), b = pair_b<Q>(lane), p = 1 + D + lane;
      double Xa[6], Xb[6];
      for (int i = 0; i < 6; ++i) { Xa[i] = Xs[1 + a][i]; Xb[i] = Xs[1 + b][i]; }
      Amul(p, X0, t1);
      for (int i = 0; i < 6; ++i) rhs[i] = -(sums[(21 + i) * NC + p] + t1[i]);
      Amul(1 + a, Xb, t1);
      Amul(1 + b, Xa, t2);
      for (int i = 0; i < 6; ++i) rhs[i] -= t1[i] + t2[i];
      solve(rhs, x);
      for (int i = 0; i < 6; ++i) Xs[p][i] = x[i];
    }
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
    for (int a = 0; a < 6; ++a)
      for (int c = 0; c < NC; ++c) dx[a].v[c] = Xs[c][a];
  }
  return true;
}

// Association, gates, residual and Jacobian of one current pixel; false if
// the pixel gives no correspondence.  J is the jet of the computation (the
// context's, or a chunk of its parts), ld(base, index) loads a 3-vector map
// entry as a J.
// kHold: the bilinear lookup's fractional position is taken from the real
// parts, so the looked-up model point and normal do not move with the jet's
// directions (the correspondences of a pass held fixed).
template <bool kHold = false, typename J, typename KP, typename LD, typename T, int D, int Q>
__device__ __forceinline__ bool icp_pixel_from(const KParams<T, D, Q>& kp, const IcpArgs<T, D, Q>& g, const KP& Tc,
                                               const KP& Tp, const J& fx, const J& fy, const J& cx, const J& cy,
                                               size_t n, uint32_t vi, const V3<J>& v, const V3<J>& nv, J jac[6], J& r,
                                               LD&& ld) {
  const int W = g.W, H = g.H;
  if (!vi) return false;
  const V3<J> p = pose_apply(Tc, v);
  const V3<J> nr = pose_rotate(Tc, nv);
  const V3<J> xc = pose_apply_inv(Tp, p);
  if (!(xc.z.re() > T(0))) return false;
  const J ux = fx * xc.x / xc.z + cx;
  const J uy = fy * xc.y / xc.z + cy;
  // tap choice floor(u + 1e-3): at the first pass of a level every pixel
  // re-projects onto its own integer coordinate up to rounding
  const T rx = ux.re(), ry = uy.re();
  const T fx0 = floor(rx + T(kTapBias)), fy0 = floor(ry + T(kTapBias));
  if (!(fx0 >= T(0) && fy0 >= T(0) && fx0 <= T(W - 2) && fy0 <= T(H - 2))) return false;
  const int i0 = int(fx0), j0 = int(fy0);
  const size_t t0 = size_t(j0) * W + i0, t1 = t0 + 1, t2 = t0 + W, t3 = t2 + 1;
  V3<J> q, m;
  if constexpr (J::N <= 8) {
    // everything the four taps hold, in flight at once; the nearest tap
    // floor(u + 1/2) is one of them (u - floor(u + 1e-3) lies in [-1e-3, 1))
    uint32_t w01 = g.validm[t0] | uint32_t(g.validm[t1]) << 8, w23 = g.validm[t2] | uint32_t(g.validm[t3]) << 8;
    T z0 = g.Zm[t0], z1 = g.Zm[t1], z2 = g.Zm[t2], z3 = g.Zm[t3];
    V3<J> q0 = ld(g.Vm, t0), q1 = ld(g.Vm, t1);
    V3<J> q2 = ld(g.Vm, t2), q3 = ld(g.Vm, t3);
    V3<J> m0 = ld(g.Nm, t0), m1 = ld(g.Nm, t1);
    V3<J> m2 = ld(g.Nm, t2), m3 = ld(g.Nm, t3);
    pin(w01);
    pin(w23);
    pin(z0);
    pin(z1);
    pin(z2);
    pin(z3);
    pin(q0);
    pin(q1);
    pin(q2);
    pin(q3);
    pin(m0);
    pin(m1);
    pin(m2);
    pin(m3);
    if (!((w01 & 0xff) && (w01 >> 8) && (w23 & 0xff) && (w23 >> 8))) return false;
    const int in = int(floor(rx + T(0.5))), jn = int(floor(ry + T(0.5)));
    const bool inside = (in == i0 || in == i0 + 1) && (jn == j0 || jn == j0 + 1);
    const int sel = (jn - j0) * 2 + (in - i0);
    const size_t tn = size_t(jn) * W + in;
    const T zn = inside ? (sel == 0 ? z0 : sel == 1 ? z1 : sel == 2 ? z2 : z3) : g.Zm[tn];
    const T disc = fabs(z0 - zn) + fabs(z1 - zn) + fabs(z2 - zn) + fabs(z3 - zn);
    if (disc >= kp.disc_delta) {
      if (inside) {
        q = sel == 0 ? q0 : sel == 1 ? q1 : sel == 2 ? q2 : q3;
        m = sel == 0 ? m0 : sel == 1 ? m1 : sel == 2 ? m2 : m3;
      } else {
        q = ld(g.Vm, tn);
        m = ld(g.Nm, tn);
      }
    } else {
      const J a = kHold ? jconst<J>(rx - fx0) : ux - fx0, b = kHold ? jconst<J>(ry - fy0) : uy - fy0;
      const J a1 = jconst<J>(T(1)) - a, b1 = jconst<J>(T(1)) - b;
      q = vadd(vscale(b1, vadd(vscale(a1, q0), vscale(a, q1))), vscale(b, vadd(vscale(a1, q2), vscale(a, q3))));
      V3<J> mm = vadd(vscale(b1, vadd(vscale(a1, m0), vscale(a, m1))), vscale(b, vadd(vscale(a1, m2), vscale(a, m3))));
      m = vscale(jconst<J>(T(1)) / jsqrt(vdot(mm, mm)), mm);
    }
  } else {
    // many components: the taps are loaded only as they are used (registers)
    if (!(g.validm[t0] && g.validm[t1] && g.validm[t2] && g.validm[t3])) return false;
    const int in = int(floor(rx + T(0.5))), jn = int(floor(ry + T(0.5)));
    const size_t tn = size_t(jn) * W + in;
    const T zn = g.Zm[tn];
    const T disc = fabs(g.Zm[t0] - zn) + fabs(g.Zm[t1] - zn) + fabs(g.Zm[t2] - zn) + fabs(g.Zm[t3] - zn);
    if (disc >= kp.disc_delta) {
      q = ld(g.Vm, tn);
      m = ld(g.Nm, tn);
    } else {
      const J a = kHold ? jconst<J>(rx - fx0) : ux - fx0, b = kHold ? jconst<J>(ry - fy0) : uy - fy0;
      const J a1 = jconst<J>(T(1)) - a, b1 = jconst<J>(T(1)) - b;
      const V3<J> q0 = ld(g.Vm, t0), q1 = ld(g.Vm, t1);
      const V3<J> q2 = ld(g.Vm, t2), q3 = ld(g.Vm, t3);
      q = vadd(vscale(b1, vadd(vscale(a1, q0), vscale(a, q1))), vscale(b, vadd(vscale(a1, q2), vscale(a, q3))));
      const V3<J> m0 = ld(g.Nm, t0), m1 = ld(g.Nm, t1);
      const V3<J> m2 = ld(g.Nm, t2), m3 = ld(g.Nm, t3);
      V3<J> mm = vadd(vscale(b1, vadd(vscale(a1, m0), vscale(a, m1))), vscale(b, vadd(vscale(a1, m2), vscale(a, m3))));
      m = vscale(jconst<J>(T(1)) / jsqrt(vdot(mm, mm)), mm);
    }
  }
  const V3<J> d = vsub(p, q);
  if (!(vdot(d, d).re() <= kp.dgate2)) return false;
  if (!(vdot(nr, m).re() >= kp.cos_agate)) return false;
  r = vdot(d, m);
  const V3<J> pm = vcross(p, m);
  jac[0] = pm.x; jac[1] = pm.y; jac[2] = pm.z; jac[3] = m.x; jac[4] = m.y; jac[5] = m.z;
  return true;
}

// the pixel's maps are loaded together with its flag (one memory round trip),
// then the rest of the pixel
template <bool kHold = false, typename J, typename KP, typename LD, typename T, int D, int Q>
__device__ __forceinline__ bool icp_pixel_with(const KParams<T, D, Q>& kp, const IcpArgs<T, D, Q>& g, const KP& Tc,
                                               const KP& Tp, const J& fx, const J& fy, const J& cx, const J& cy,
                                               size_t n, size_t i, J jac[6], J& r, LD&& ld) {
  uint32_t vi = g.valid[i];
  V3<J> v = ld(g.V, i), nv = ld(g.N, i);
  pin(vi);
  pin(v);
  pin(nv);
  return icp_pixel_from<kHold>(kp, g, Tc, Tp, fx, fy, cx, cy, n, vi, v, nv, jac, r, ld);
}

template <typename T, int D, int Q>
__device__ __forceinline__ bool icp_pixel(const KParams<T, D, Q>& kp, const IcpArgs<T, D, Q>& g,
                                          const KPose<T, D, Q>& Tc, const KPose<T, D, Q>& Tp,
                                          const Jet<T, D, Q>& fx, const Jet<T, D, Q>& fy, const Jet<T, D, Q>& cx,
                                          const Jet<T, D, Q>& cy, size_t n, size_t i, Jet<T, D, Q> jac[6],
                                          Jet<T, D, Q>& r) {
  return icp_pixel_with(kp, g, Tc, Tp, fx, fy, cx, cy, n, i, jac, r,
                        [&](const T* base, size_t idx) { return vload<Jet<T, D, Q>>(base, n, idx); });
}

// Parts of a chunk of a jet: part 0 is the real part, parts 1..Dc are the
// directions d0..d0+Dc-1 of the full jet (D directions, Q pair directions),
// and a chunk with Qc = Q (then d0 = 0, Dc >= Q) also holds the Q(Q+1)/2 pair
// parts.  Every part of a chunk is computed with the arithmetic it has in the
// full jet (a product's part c needs parts 0 and c, a pair part also the parts
// of its two directions, all in the same chunk).
template <int D, int Q, int Dc, int Qc, int d0>
struct SubParts {
  static_assert(Qc == 0 || (Qc == Q && d0 == 0 && Dc >= Q), "pairs need their directions");
  static constexpr int NF = 1 + D + Q * (Q + 1) / 2;
  __host__ __device__ static constexpr int at(int c) { return c == 0 ? 0 : (c <= Dc ? d0 + c : 1 + D + (c - 1 - Dc)); }
};
template <typename SP, typename T, int D, int Q, int Dc, int Qc>
__device__ __forceinline__ void jsub(const Jet<T, D, Q>& x, Jet<T, Dc, Qc>& y) {
#pragma unroll
  for (int c = 0; c < Jet<T, Dc, Qc>::N; ++c) y.v[c] = x.v[SP::at(c)];
}
template <typename F, int... JJ>
__device__ __forceinline__ void for_each_index(F&& f, std::integer_sequence<int, JJ...>) {
  (f(std::integral_constant<int, JJ>{}), ...);
}
// ICP chunk plan for many parts: chunk 0 holds the pair directions and the
// pairs (or 6 directions when there are no pairs), then 6 directions each
template <int D, int Q>
struct IcpChunks {
  static constexpr int D0 = Q > 0 ? Q : (D < 6 ? D : 6);
  static constexpr int count = 1 + (D - D0 + 5) / 6;
  static constexpr int start(int j) { return j == 0 ? 0 : D0 + 6 * (j - 1); }
  static constexpr int dirs(int j) { return j == 0 ? D0 : (D - start(j) < 6 ? D - start(j) : 6); }
  static constexpr int pairs(int j) { return j == 0 ? Q : 0; }
};

// Per-block sums of the normal equations of one ICP pass (21 entries of
// A = sum J J^T, 6 of b = sum J r, each with NC components; count; sum r^2).
// Few components: per-thread sums over a few pixels, then an FP64 block tree.
// Many components: every pixel's terms are reduced across the wave at once
// (FP64) into per-wave LDS accumulators, so no thread holds 27 NC sums.
// The solve after the sums (one wave): FP64 solve, relaxation, SE(3) update
// (one entry of the new pose per lane), counters; or only the sums when they
// are all that is wanted.
//
// What the finish needs from memory besides the sums, loaded by the solving
// wave when the kernel starts, so that these round trips overlap the sums'
// instead of following the solve one after another: the frame's counter row
// (and the two counters it reads back), and lane (r, c)'s column of the pose.
// (Jets of up to 8 parts, the 1024-thread finish; the many-part finish keeps
// these loads where they are used: holding them from the start there added
// spills to a kernel that already keeps most of its state in scratch, and
// the 16 + 10 shape then lost its tangents.)
template <typename T, int D, int Q>
constexpr bool kFinishPreload = Jet<T, D, Q>::N <= 8;
template <int D, int Q>
struct FinishPre {
  int32_t* crow;
  int32_t crow3, crow32;
  Jet<double, D, Q> col[3];
};
template <typename T, int D, int Q>
__device__ __forceinline__ FinishPre<D, Q> finish_preload(const IcpArgs<T, D, Q>& g, int lane) {
  FinishPre<D, Q> pre;
  const int c = lane & 3;
  if (lane < 12) pose_column<D, Q>(g.Pcur, c, pre.col);
  pre.crow = counter_row(g.counters, g.frame, g.max_frames);
  pre.crow3 = 0;
  pre.crow32 = 0;
  if (g.do_solve && lane == 0) {
    pre.crow3 = pre.crow[3];
    pre.crow32 = pre.crow[32];
  }
  return pre;
}

template <typename T, int D, int Q>
__device__ void icp_finish_solve(const IcpArgs<T, D, Q>& g, const double* fin, int lane, double (*Xs)[6],
                                 const FinishPre<D, Q>& pre) {
  constexpr int NC = Jet<T, D, Q>::N;
  constexpr int NS = IcpSize<D, Q>::NS;
  constexpr bool kPre = kFinishPreload<T, D, Q>;
  const int cnt = int(fin[27 * NC]);
  int32_t* crow = kPre ? pre.crow : counter_row(g.counters, g.frame, g.max_frames);
  if (!g.do_solve) {
    for (int k = lane; k < NS; k += 64) g.sums_out[k] = fin[k];
    return;
  }
  if (lane == 0) {
    crow[3] = (kPre ? pre.crow3 : crow[3]) + cnt;
    crow[4] = cnt;
    if (g.iter_slot < kMaxPasses) crow[5 + g.iter_slot] = cnt;
  }
  // every lane solves (the same operations on the same data), so the update
  // is known to all of them without a broadcast
  Jet<double, D, Q> dx[6];
  if (cnt < 6 || !icp_solve<D, Q>(fin, dx, lane, Xs)) {
    if (lane == 0) {
      *g.lost = 1;
      crow[0] = 1;
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) dx[a] = g.omega * dx[a];
  if (lane == 0) {
    double nn = 0.0;
    for (int a = 0; a < 6; ++a) nn += dx[a].re() * dx[a].re();
    if ((kPre ? pre.crow32 : crow[32]) == 0 && sqrt(nn) < 1e-6) crow[32] = g.iter_slot + 1;
  }
  // the update exp(dx) * P, one of its 12 entries per lane
  if (lane >= 12) return;
  const int r = lane >> 2, c = lane & 3;
  Jet<double, D, Q> e;
  if constexpr (kPre)
    e = g.update ? smallangle_mul_entry<D, Q>(dx, pre.col, r, c) : se3_exp_mul_entry<D, Q>(dx, pre.col, r, c);
  else
    e = g.update ? smallangle_mul_entry<D, Q>(dx, g.Pcur, r, c) : se3_exp_mul_entry<D, Q>(dx, g.Pcur, r, c);
  if (g.update) {
    // the composed rotation back to orthonormal: every lane gathers the nine
    // rotation entries and runs the same two polar Newton steps on them
    using JD = Jet<double, D, Q>;
    __shared__ JD Rsh[9];
    if (c < 3) Rsh[r * 3 + c] = e;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    JD R[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) R[q] = Rsh[q];
    polar_steps<D, Q>(R);
    if (c < 3) e = R[r * 3 + c];
  }
  // (every lane has read its column of P: the lanes of one wave issue their
  // loads together, before any of them stores)
  __builtin_amdgcn_wave_barrier();
  const int idx = c < 3 ? r * 3 + c : 9 + r;
  g.Pcur->m[idx] = e;
  Jet<T, D, Q>* ke = c < 3 ? &g.Kcur->R[r * 3 + c] : &g.Kcur->t[r];
  *ke = jcast<T>(e);
}


template <typename T, int D, int Q>
__device__ __forceinline__ void icp_body(const VB& vb, const KParams<T, D, Q>& kp, const IcpArgs<T, D, Q>& g) {
  using J = Jet<T, D, Q>;
  constexpr int NC = J::N;
  constexpr int NS = IcpSize<D, Q>::NS;
  constexpr bool kRegAcc = NS <= 192;
  constexpr bool kPrefetch = NC <= 2;   // registers for the next pixel's maps
  __shared__ double red[kIcpThreads / 64][NS];
  // (no test of the lost flag here: after a lost pass the pose is left as it
  // was, these sums are computed from it and k_icp_finish drops them; a test
  // would put one more memory round trip before the first pixel of every pass)
  const KPose<T, D, Q> Tc = *g.Kcur;
  const KPose<T, D, Q> Tp = *g.Kprev;
  const T sc = T(1) / T(1 << g.level);
  const J fx = kp.fx * sc, fy = kp.fy * sc, cx = kp.cx * sc, cy = kp.cy * sc;
  const size_t n = size_t(g.W) * g.H;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // each logical workgroup takes a contiguous run of pixels (a multiple of the
  // workgroup size); with the XCD remap every L2 sees one band of the image
  const size_t chunk = (n + size_t(vb.gx) * kIcpThreads - 1) / (size_t(vb.gx) * kIcpThreads) * kIcpThreads;
  const size_t p0 = size_t(xcd_remap(vb.bx, vb.gx)) * chunk;
  const size_t p1 = p0 + chunk < n ? p0 + chunk : n;

  if constexpr (kRegAcc) {
    T acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0;
    auto accumulate = [&](const J (&jac)[6], const J& r) {
      int k = 0;
#pragma unroll
      for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = a; b < 6; ++b, ++k) {
          const J prod = jac[a] * jac[b];
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[k * NC + c] += prod.v[c];
        }
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const J prod = jac[a] * r;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[(21 + a) * NC + c] += prod.v[c];
      }
      acc[27 * NC] += T(1);
      acc[27 * NC + 1] += r.re() * r.re();
    };
    if constexpr (kPrefetch) {
      // Each thread's pixels are taken one after the other; the maps of its
      // next pixel are loaded before the current one's model taps, so that the
      // two memory round trips of consecutive pixels overlap (the sums and
      // their order are those of one pixel at a time).
      auto ld = [&](const T* base, size_t idx) { return vload<J>(base, n, idx); };
      size_t i = p0 + threadIdx.x;
      uint32_t vi = 0;
      V3<J> v{}, nv{};
      if (i < p1) {
        vi = g.valid[i];
        v = ld(g.V, i);
        nv = ld(g.N, i);
      }
      for (; i < p1; i += kIcpThreads) {
        uint32_t vi2 = 0;
        V3<J> v2 = v, nv2 = nv;
        if (i + kIcpThreads < p1) {
          vi2 = g.valid[i + kIcpThreads];
          v2 = ld(g.V, i + kIcpThreads);
          nv2 = ld(g.N, i + kIcpThreads);
        }
        pin(vi);
        pin(v);
        pin(nv);
        J jac[6], r;
        const bool ok = icp_pixel_from(kp, g, Tc, Tp, fx, fy, cx, cy, n, vi, v, nv, jac, r, ld);
        vi = vi2;
        v = v2;
        nv = nv2;
        if (ok) accumulate(jac, r);
      }
    } else {
      for (size_t i = p0 + threadIdx.x; i < p1; i += kIcpThreads) {
        J jac[6], r;
        if (icp_pixel(kp, g, Tc, Tp, fx, fy, cx, cy, n, i, jac, r)) accumulate(jac, r);
      }
    }
    // block reduction in FP64: wave butterflies, then the 4 waves in fixed
    // order.  The tangent sums cancel strongly (the derivative of a converged
    // pose is a small difference of large per-pixel terms), so only the
    // per-thread sums over a few pixels stay in T.
    {
      constexpr int M = (NS + 63) / 64;
      double tot[M];
      wave_sum_transposed<NS>(acc, lane, tot);
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (lane * M + j < NS) red[wv][lane * M + j] = tot[j];
    }
  } else {
    // real components (and count, sum r^2) exactly as in the register path, so
    // real parts do not depend on the number of components; the others are
    // reduced across the wave pixel by pixel
    T racc[29];
#pragma unroll
    for (int k = 0; k < 29; ++k) racc[k] = 0;
    for (int k = lane; k < NS; k += 64) red[wv][k] = 0.0;
    // The pixel is evaluated chunk by chunk of the jet's parts (each chunk's
    // jets fit in registers; the real part is recomputed, identically, in
    // every chunk and accumulated from the first); every part keeps the
    // arithmetic and summation order it has in the full jet.
    using CP = IcpChunks<D, Q>;
    auto chunk = [&](auto ji, size_t i, T (&ra)[29]) {
      constexpr int j = decltype(ji)::value;
      constexpr int Dc = CP::dirs(j), Qc = CP::pairs(j), d0 = CP::start(j);
      using SP = SubParts<D, Q, Dc, Qc, d0>;
      using JC = Jet<T, Dc, Qc>;
      KPose<T, Dc, Qc> Tcc, Tpc;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        jsub<SP>(Tc.R[q], Tcc.R[q]);
        jsub<SP>(Tp.R[q], Tpc.R[q]);
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        jsub<SP>(Tc.t[q], Tcc.t[q]);
        jsub<SP>(Tp.t[q], Tpc.t[q]);
      }
      JC fxc, fyc, cxc, cyc;
      jsub<SP>(fx, fxc);
      jsub<SP>(fy, fyc);
      jsub<SP>(cx, cxc);
      jsub<SP>(cy, cyc);
      auto ld = [&](const T* b, size_t idx) {
        V3<JC> v;
        JC* o[3] = {&v.x, &v.y, &v.z};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int c = 0; c < JC::N; ++c) o[a]->v[c] = b[size_t(a * NC + SP::at(c)) * n + idx];
        return v;
      };
      JC jac[6], r;
      const bool ok = i < p1 && icp_pixel_with(kp, g, Tcc, Tpc, fxc, fyc, cxc, cyc, n, i, jac, r, ld);
      if (!ok) {
        r = jzero<JC>();
#pragma unroll
        for (int a = 0; a < 6; ++a) jac[a] = jzero<JC>();
      }
      if constexpr (j == 0) {
        if (ok) {
          int k = 0;
#pragma unroll
          for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int b = a; b < 6; ++b, ++k) ra[k] += jac[a].v[0] * jac[b].v[0];
#pragma unroll
          for (int a = 0; a < 6; ++a) ra[21 + a] += jac[a].v[0] * r.v[0];
          ra[27] += T(1);
          ra[28] += r.re() * r.re();
        }
      }
      constexpr int NCHK = (27 * (JC::N - 1) + 63) / 64;
      icp_tangent_sums<T, Dc, Qc, NC, SP>(jac, r, lane, red[wv], std::make_integer_sequence<int, NCHK>{});
    };
    for (size_t base = p0; base < p1; base += kIcpThreads) {
      const size_t i = base + threadIdx.x;
      if constexpr (CP::count > 1) {
        for_each_index([&](auto ji) { chunk(ji, i, racc); }, std::make_integer_sequence<int, CP::count>{});
      } else {
        J jac[6], r;
        const bool ok = i < p1 && icp_pixel(kp, g, Tc, Tp, fx, fy, cx, cy, n, i, jac, r);
        if (!ok) {
          r = jzero<J>();
#pragma unroll
          for (int a = 0; a < 6; ++a) jac[a] = jzero<J>();
        }
        if (ok) {
          int k = 0;
#pragma unroll
          for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int b = a; b < 6; ++b, ++k) racc[k] += jac[a].v[0] * jac[b].v[0];
#pragma unroll
          for (int a = 0; a < 6; ++a) racc[21 + a] += jac[a].v[0] * r.v[0];
        }
        constexpr int NCH = (27 * (NC - 1) + 63) / 64;
        icp_tangent_sums<T, D, Q>(jac, r, lane, red[wv], std::make_integer_sequence<int, NCH>{});
        if (ok) {
          racc[27] += T(1);
          racc[28] += r.re() * r.re();
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      const double sv = wave_sum(double(racc[k]));
      if (lane == 0) red[wv][k * NC] = sv;
    }
    const double sc1 = wave_sum(double(racc[27])), sr2 = wave_sum(double(racc[28]));
    if (lane == 0) { red[wv][27 * NC] = sc1; red[wv][27 * NC + 1] = sr2; }
  }
  __syncthreads();
  double* part = g.partials + size_t(vb.bx) * NS;
  for (int k = threadIdx.x; k < NS; k += kIcpThreads) {
    double s = red[0][k];
#pragma unroll
    for (int w = 1; w < kIcpThreads / 64; ++w) s += red[w][k];
    part[k] = s;
  }
}
template <typename T, int D, int Q>
__global__ __launch_bounds__(kIcpThreads) void k_icp(KParams<T, D, Q> kp, IcpArgs<T, D, Q> g) {
  icp_body<T, D, Q>(VB::hw(), kp, g);
}

// One workgroup after k_icp (a kernel boundary makes every partial visible to
// it without device-wide fences in k_icp, whose cross-XCD L2 write-back cost
// more than the launch it would save).  Each component is summed over the
// workgroup partials in the same order whatever the number of components (so
// real parts do not depend on D, Q): 16 interleaved groups of workgroups
// (b mod 16), eight running sums each, combined in a fixed tree; components
// are taken 64 at a time, one (component, group) per thread (1024 threads),
// or four groups per thread for jets with many parts (256 threads, so that
// the solving wave may hold 512 registers: the same sums, fewer spills).
template <typename T, int D, int Q>
constexpr int kFinishThreads = Jet<T, D, Q>::N > 2 ? 256 : 1024;
template <typename T, int D, int Q>
__device__ __forceinline__ void icp_finish_body(const VB& vb, const IcpArgs<T, D, Q>& g, int nblocks) {
  constexpr int NS = IcpSize<D, Q>::NS;
  constexpr int NT = kFinishThreads<T, D, Q>;
  constexpr int G = 16, KC = 64, GPT = G * KC / NT;
  __shared__ double gs[G][KC];
  __shared__ double fin[NS];
  __shared__ double xs[Jet<T, D, Q>::N][6];
  const int lost = *g.lost;   // read now, tested after the sums (its load overlaps theirs)
  FinishPre<D, Q> pre;
  if constexpr (kFinishPreload<T, D, Q>)
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
        // the m-th workgroup of the group (b = grp + m G) goes to running sum
        // m mod 8, in increasing m; its partials are loaded NB at a time with
        // every load in flight together (indexes past the end are clamped and
        // their values dropped)
        constexpr unsigned NB = 32;
        for (unsigned b0 = grp; b0 < B; b0 += NB * G) {
          double v[NB];
#pragma unroll
          for (unsigned u = 0; u < NB; ++u) {
            const unsigned b = b0 + u * G < B ? b0 + u * G : B - 1;
            v[u] = g.partials[size_t(b) * NS + k];
          }
#pragma unroll
          for (unsigned u = 0; u < NB; ++u)
            if (b0 + u * G < B) a8[u & 7] += v[u];
        }
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
  icp_finish_solve<T, D, Q>(g, fin, threadIdx.x, xs, pre);
}
template <typename T, int D, int Q>
__global__ __launch_bounds__((kFinishThreads<T, D, Q>)) void k_icp_finish(IcpArgs<T, D, Q> g, int nblocks) {
  icp_finish_body<T, D, Q>(VB::hw(), g, nblocks);
}


// start of tracking for frame k >= 1: shift the pose history and set the
// initial estimate: the previous pose, or constant velocity T1 T2^-1 T1 when
// both previous frames were tracked (after a lost frame the velocity is
// unknown, and extrapolating a guess would never re-acquire the camera)
template <typename T, int D, int Q>
struct TrackBegin {
  MPose<D, Q>* Pcur;
  MPose<D, Q>* Pprev;
  MPose<D, Q>* Pprev2;
  MPose<D, Q>* Pinit;
  KPose<T, D, Q>* Kcur;
  KPose<T, D, Q>* Kprev;
  int* lost;                // nullptr: nothing to do
  int32_t* counter_base;
  const int* frame;
  int max_frames;
  int const_vel;
};
template <typename T, int D, int Q>
__device__ void track_begin_work(const TrackBegin<T, D, Q>& a) {
  int32_t* counters = counter_row(a.counter_base, a.frame, a.max_frames);
  *a.Pprev2 = *a.Pprev;
  *a.Pprev = *a.Pcur;
  MPose<D, Q> init = *a.Pprev;
  const int k = *a.frame;
  const int max_frames = a.max_frames;
  int32_t* counter_base = a.counter_base;
  if (a.const_vel && k > 1 && k - 1 < max_frames) {
    const bool tracked = counter_base[size_t(kCounters) * (k - 1)] == 0 && counter_base[size_t(kCounters) * (k - 2)] == 0;
    if (tracked) {
      init = pose_mul(*a.Pprev, pose_mul(pose_inverse(*a.Pprev2), *a.Pprev));
      // R1 R2^T R1 triples the rotation's departure from orthonormality, and
      // the next prediction starts from it: two Newton steps of the polar
      // decomposition keep it at rounding level
      polar_steps<D, Q>(init.m);
    }
  }
  *a.Pinit = init;
  *a.Pcur = init;
  *a.Kcur = to_kpose<T, double>(init);
  *a.Kprev = to_kpose<T, double>(*a.Pprev);
  *a.lost = 0;
  for (int i = 0; i < kCounters; ++i) counters[i] = 0;
}
template <typename T, int D, int Q>
__global__ void k_track_begin(TrackBegin<T, D, Q> a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  track_begin_work(a);
}

// ---------------------------------------------------------------------------
// A6. TSDF fusion (Sec. 4.1 "Surface Update"), one workgroup per 8^3 brick.
// ---------------------------------------------------------------------------
template <typename T, int D, int Q>
__device__ __forceinline__ void voxel_centre(const KParams<T, D, Q>& kp, int i, int j, int k, T c[3]) {
  const double s = double(kp.voxel);
  c[0] = T((i + 0.5) * s - 0.5 * kp.dim[0] * s);
  c[1] = T((j + 0.5) * s - 0.5 * kp.dim[1] * s);
  c[2] = T((k + 0.5) * s - 0.5 * kp.dim[2] * s);
}

// Largest filtered depth per 16x16 tile of level 0 (bound of every L(x)
// whose bilinear taps fall in that tile).
constexpr int kTile = 16;
// Largest filtered depth of every 16x16 tile of level 0 (tmax) and of every
// 64x64 cell of 4x4 tiles (cmax): one workgroup per cell, 16 lanes per tile,
// each lane one tile row.
constexpr int kCell = 4;   // tiles per coarse cell and axis

// End of tracking (a lost frame keeps its initial estimate), pose history, and
// the reset of the brick list for fusion; one thread.
template <typename T, int D, int Q>
struct PostTrack {
  MPose<D, Q>* Pcur;
  const MPose<D, Q>* Pinit;
  KPose<T, D, Q>* Kcur;
  const int* lost;        // nullptr: the frame was not tracked
  MPose<D, Q>* history;   // nullptr: no history entry
  const int* frame;
  int max_frames;
  int* count;
};
template <typename T, int D, int Q>
__device__ void post_track_work(const PostTrack<T, D, Q>& a) {
  if (a.lost && *a.lost) {
    *a.Pcur = *a.Pinit;
    *a.Kcur = to_kpose<T, double>(*a.Pinit);
  }
  if (a.history) a.history[min(*a.frame, a.max_frames - 1)] = *a.Pcur;
  *a.count = 0;
}

// (post.count != nullptr: workgroup 0 also does the end-of-tracking work, which
// the kernels after this one read)
template <typename T, int D, int Q>
__device__ __forceinline__ void tile_zmax_body(const VB& vb, const T* __restrict__ D0, int W, int H, T* __restrict__ tmax,
                                                             T* __restrict__ cmax, const PostTrack<T, D, Q>& post) {
  if (post.count && vb.bx == 0 && vb.by == 0 && threadIdx.x == 0) post_track_work(post);
  const int ntx = (W + kTile - 1) / kTile, nty = (H + kTile - 1) / kTile;
  const int tile = threadIdx.x >> 4, row = threadIdx.x & 15;
  const int tx = vb.bx * kCell + (tile & 3), ty = vb.by * kCell + (tile >> 2);
  T m = 0;
  const int y = ty * kTile + row;
  if (tx < ntx && ty < nty && y < H) {
    const T* src = D0 + size_t(y) * W;
#pragma unroll
    for (int i = 0; i < kTile; ++i) {
      const int x = tx * kTile + i;
      if (x < W) {
        const T d = src[x];
        m = d > m ? d : m;
      }
    }
  }
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) { const T v = __shfl_xor(m, o, 64); m = v > m ? v : m; }
  if (row == 0 && tx < ntx && ty < nty) tmax[ty * ntx + tx] = m;
#pragma unroll
  for (int o = 32; o >= 16; o >>= 1) { const T v = __shfl_xor(m, o, 64); m = v > m ? v : m; }
  __shared__ T wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const T a = wm[0] > wm[1] ? wm[0] : wm[1], b = wm[2] > wm[3] ? wm[2] : wm[3];
    cmax[vb.by * vb.gx + vb.bx] = a > b ? a : b;
  }
}
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_tile_zmax(const T* __restrict__ D0, int W, int H, T* __restrict__ tmax,
                                                   T* __restrict__ cmax, PostTrack<T, D, Q> post) {
  tile_zmax_body<T, D, Q>(VB::hw(), D0, W, H, tmax, cmax, post);
}

// Whether brick b may hold a voxel that fusion at the pose P (real parts)
// updates (a conservative sphere test): in front of the camera, intersecting
// the four frustum planes of the pixel range that admits a bilinear depth
// lookup, and not farther than mu behind the largest depth over the tiles its
// projection (plus one pixel) covers.
template <typename T, int D, int Q>
__device__ __forceinline__ bool brick_may_update(const KParams<T, D, Q>& kp, const KPose<T, D, Q>& P,
                                                 const T* __restrict__ tmax, const T* __restrict__ cmax, int b) {
  const int bx = b % kp.nbr[0], by = (b / kp.nbr[0]) % kp.nbr[1], bz = b / (kp.nbr[0] * kp.nbr[1]);
  const double s = double(kp.voxel);
  const double c[3] = {(bx * 8 + 4) * s - 0.5 * kp.dim[0] * s, (by * 8 + 4) * s - 0.5 * kp.dim[1] * s,
                       (bz * 8 + 4) * s - 0.5 * kp.dim[2] * s};
  const double r = 4.0 * 1.7320508075688772 * s * 1.01;
  double d[3], x[3];
  for (int a = 0; a < 3; ++a) d[a] = c[a] - double(P.t[a].re());
  for (int a = 0; a < 3; ++a)
    x[a] = double(P.R[0 + a].re()) * d[0] + double(P.R[3 + a].re()) * d[1] + double(P.R[6 + a].re()) * d[2];
  const double fx = kp.fx.re(), fy = kp.fy.re(), cx = kp.cx.re(), cy = kp.cy.re();
  const double n[4][3] = {{fx, 0, cx}, {-fx, 0, double(kp.W - 1) - cx}, {0, fy, cy}, {0, -fy, double(kp.H - 1) - cy}};
  bool keep = x[2] + r > 0.0;
  for (int q = 0; q < 4 && keep; ++q) {
    const double dn = n[q][0] * x[0] + n[q][1] * x[1] + n[q][2] * x[2];
    const double nn = sqrt(n[q][0] * n[q][0] + n[q][1] * n[q][1] + n[q][2] * n[q][2]);
    keep = dn >= -r * nn;
  }
  // a brick reaching to the camera plane (z0 <= 1 mm) has no bounded
  // footprint: it is kept without the depth test (a conservative cull)
  if (keep && x[2] - r > 1e-3) {
    const int ntx = (kp.W + kTile - 1) / kTile;
    int tx0, tx1, ty0, ty1;
    const double z0 = x[2] - r, z1 = x[2] + r;
    {
      const double ul = cx + fx * fmin((x[0] - r) / z0, (x[0] - r) / z1), uh = cx + fx * fmax((x[0] + r) / z0, (x[0] + r) / z1);
      const double vl = cy + fy * fmin((x[1] - r) / z0, (x[1] - r) / z1), vh = cy + fy * fmax((x[1] + r) / z0, (x[1] + r) / z1);
      const int pxl = int(fmax(floor(ul) - 1.0, 0.0)), pxh = int(fmin(floor(uh) + 2.0, double(kp.W - 1)));
      const int pyl = int(fmax(floor(vl) - 1.0, 0.0)), pyh = int(fmin(floor(vh) + 2.0, double(kp.H - 1)));
      tx0 = pxl / kTile; tx1 = pxh / kTile; ty0 = pyl / kTile; ty1 = pyh / kTile;
    }
    double zm = 0.0;
    if ((tx1 - tx0 + 1) * (ty1 - ty0 + 1) <= kCell * kCell) {
      for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) zm = fmax(zm, double(tmax[ty * ntx + tx]));
    } else {
      // a large footprint: the 64x64 cells covering it (a bound at least as large)
      const int ncx = (ntx + kCell - 1) / kCell;
      for (int cy = ty0 / kCell; cy <= ty1 / kCell; ++cy)
        for (int cx = tx0 / kCell; cx <= tx1 / kCell; ++cx) zm = fmax(zm, double(cmax[cy * ncx + cx]));
    }
    keep = zm > 0.0 && z0 <= zm + double(kp.mu.re()) * 1.01 + 1e-6;
  }
  return keep;
}

// The bricks fusion at the current pose may update, appended to a list.
template <typename T, int D, int Q>
__device__ __forceinline__ void brick_cull_body(const VB& vb, const KParams<T, D, Q>& kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                              const T* __restrict__ tmax, const T* __restrict__ cmax,
                                                              int nbrick, int* __restrict__ list,
                                                              int* __restrict__ count, const int* __restrict__ lost) {
  const int b = vb.bx * 256 + threadIdx.x;
  const bool keep = b < nbrick && !*lost && brick_may_update(kp, *Kk, tmax, cmax, b);
  // one list append per workgroup (ballots, then a prefix over the 4 waves)
  const unsigned long long bal = __ballot(keep);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ int wcount[4], wbase[4], bbase;
  if (lane == 0) wcount[wv] = int(__popcll(bal));
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < 4; ++w) {
      wbase[w] = tot;
      tot += wcount[w];
    }
    bbase = tot ? atomicAdd(count, tot) : 0;
  }
  __syncthreads();
  if (keep) list[bbase + wbase[wv] + __popcll(bal & ((1ull << lane) - 1ull))] = b;
}
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_brick_cull(KParams<T, D, Q> kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                    const T* __restrict__ tmax, const T* __restrict__ cmax,
                                                    int nbrick, int* __restrict__ list,
                                                    int* __restrict__ count, const int* __restrict__ lost) {
  brick_cull_body<T, D, Q>(VB::hw(), kp, Kk, tmax, cmax, nbrick, list, count, lost);
}

template <typename T, int D, int Q>
__device__ __forceinline__ int fuse_brick(const KParams<T, D, Q>& kp, const KPose<T, D, Q>* __restrict__ Kk,
                                          const T* __restrict__ Df, typename Vec2<T>::type* __restrict__ rec,
                                          T* __restrict__ Ftan, T* __restrict__ Wtan, int64_t nvox, int b) {
  using J = Jet<T, D, Q>;
  using R0 = Jet<T, 0, 0>;
  const int t = threadIdx.x;
  const int bx = b % kp.nbr[0], by = (b / kp.nbr[0]) % kp.nbr[1], bz = b / (kp.nbr[0] * kp.nbr[1]);
  const int i = bx * 8 + (t & 7), j = by * 8 + ((t >> 3) & 7), k = bz * 8 + (t >> 6);
  const int64_t vi = int64_t(b) * kBrickVox + t;
  const int W = kp.W, H = kp.H;
  const size_t n = size_t(W) * H;
  T cc[3];
  voxel_centre(kp, i, j, k, cc);

  // ---- decisions on real parts
  const KPose<T, D, Q>& P = *Kk;
  KPose<T, 0, 0> Pr;
#pragma unroll
  for (int q = 0; q < 9; ++q) Pr.R[q].v[0] = P.R[q].re();
#pragma unroll
  for (int q = 0; q < 3; ++q) Pr.t[q].v[0] = P.t[q].re();
  const V3<R0> cr = {jconst<R0>(cc[0]), jconst<R0>(cc[1]), jconst<R0>(cc[2])};
  const V3<R0> xr = pose_apply_inv(Pr, cr);
  bool upd = false;
  int i0 = 0, j0 = 0;
  bool nearest = false;
  int sel = 0;
  T ux_r = 0, uy_r = 0;
  if (xr.z.re() > T(0)) {
    ux_r = kp.fx.re() * xr.x.re() / xr.z.re() + kp.cx.re();
    uy_r = kp.fy.re() * xr.y.re() / xr.z.re() + kp.cy.re();
    const T fx0 = floor(ux_r), fy0 = floor(uy_r);
    if (fx0 >= T(0) && fy0 >= T(0) && fx0 <= T(W - 2) && fy0 <= T(H - 2)) {
      i0 = int(fx0);
      j0 = int(fy0);
      const size_t t0 = size_t(j0) * W + i0;
      const T d0 = Df[t0], d1 = Df[t0 + 1], d2 = Df[t0 + W], d3 = Df[t0 + W + 1];
      if (d0 > T(0) && d1 > T(0) && d2 > T(0) && d3 > T(0)) {
        // the nearest pixel floor(u + 1/2) is one of the four taps (u lies in
        // [floor(u), floor(u) + 1)), so its depth is already loaded
        const int in = int(floor(ux_r + T(0.5))), jn = int(floor(uy_r + T(0.5)));
        sel = (jn - j0) * 2 + (in - i0);
        const T dn = sel == 0 ? d0 : sel == 1 ? d1 : sel == 2 ? d2 : d3;
        const T disc = fabs(d0 - dn) + fabs(d1 - dn) + fabs(d2 - dn) + fabs(d3 - dn);
        T L;
        if (disc >= kp.disc_delta) {
          nearest = true;
          L = dn;
        } else {
          const T a = ux_r - fx0, bb = uy_r - fy0;
          const T a1 = T(1) - a, b1 = T(1) - bb;
          L = b1 * (a1 * d0 + a * d1) + bb * (a1 * d2 + a * d3);
        }
        const T eta = L - xr.z.re();
        upd = !(eta < -kp.mu.re());
      }
    }
  }
  const int nupd = __syncthreads_count(upd);
  if (!upd) return nupd;

  // ---- the update in complex-step arithmetic
  // the four depth taps with their parts (the nearest is one of them) and
  // the voxel's record, all in flight together
  const size_t t0 = size_t(j0) * W + i0;
  J q0 = jload<J>(Df, n, t0), q1 = jload<J>(Df, n, t0 + 1);
  J q2 = jload<J>(Df, n, t0 + W), q3 = jload<J>(Df, n, t0 + W + 1);
  auto r = rec[vi];
  J F;
#pragma unroll
  for (int q = 1; q < J::N; ++q) F.v[q] = Ftan[size_t(q - 1) * nvox + vi];
  T wt = Wtan != nullptr ? Wtan[vi] : T(0);
  pin(q0);
  pin(q1);
  pin(q2);
  pin(q3);
  pin(r.x);
  pin(r.y);
#pragma unroll
  for (int q = 1; q < J::N; ++q) pin(F.v[q]);
  pin(wt);
  F.v[0] = r.x;
  const V3<J> c = {jconst<J>(cc[0]), jconst<J>(cc[1]), jconst<J>(cc[2])};
  const V3<J> x = pose_apply_inv(P, c);
  const J ux = kp.fx * x.x / x.z + kp.cx;
  const J uy = kp.fy * x.y / x.z + kp.cy;
  J L;
  if (nearest) {
    L = sel == 0 ? q0 : sel == 1 ? q1 : sel == 2 ? q2 : q3;
  } else {
    const J a = ux - T(i0), bb = uy - T(j0);
    const J a1 = jconst<J>(T(1)) - a, b1 = jconst<J>(T(1)) - bb;
    L = b1 * (a1 * q0 + a * q1) + bb * (a1 * q2 + a * q3);
  }
  const J eta = L - x.z;
  const J Fd = (eta.re() >= kp.mu.re()) ? jconst<J>(T(1)) : eta / kp.mu;
  J Wj = jconst<J>(r.y);
  if (Wtan != nullptr) {
#pragma unroll
    for (int q = 0; q < D; ++q)
      if (q == kp.wcap_dir) Wj.v[1 + q] = wt;
  }
  const J Fn = (Wj * F + Fd) / (Wj + T(1));
  const J Wn = (Wj.re() + T(1) < kp.wcap.re()) ? Wj + T(1) : kp.wcap;
  r.x = Fn.v[0];
  r.y = Wn.v[0];
  rec[vi] = r;
#pragma unroll
  for (int q = 1; q < J::N; ++q) Ftan[size_t(q - 1) * nvox + vi] = Fn.v[q];
  if (Wtan != nullptr) {
    T wt = 0;
#pragma unroll
    for (int q = 0; q < D; ++q)
      if (q == kp.wcap_dir) wt = Wn.v[1 + q];
    Wtan[vi] = wt;
  }
  return nupd;
}

template <typename T, int D, int Q>
__device__ __forceinline__ void fuse_body(const VB& vb, const KParams<T, D, Q>& kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                        const T* __restrict__ Df, typename Vec2<T>::type* __restrict__ rec,
                                                        T* __restrict__ Ftan, T* __restrict__ Wtan,
                                                        const int* __restrict__ lost, int64_t nvox,
                                                        const int* __restrict__ list, const int* __restrict__ count,
                                                        int* __restrict__ block_counts) {
  int total = 0;
  if (!*lost) {
    const int nact = *count;
    for (int q = vb.bx; q < nact; q += vb.gx)
      total += fuse_brick(kp, Kk, Df, rec, Ftan, Wtan, nvox, list[q]);
  }
  if (threadIdx.x == 0) block_counts[vb.bx] = total;   // summed by k_sum_counts, no atomics
}
template <typename T, int D, int Q>
__global__ __launch_bounds__(kBrickVox) void k_fuse(KParams<T, D, Q> kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                    const T* __restrict__ Df, typename Vec2<T>::type* __restrict__ rec,
                                                    T* __restrict__ Ftan, T* __restrict__ Wtan,
                                                    const int* __restrict__ lost, int64_t nvox,
                                                    const int* __restrict__ list, const int* __restrict__ count,
                                                    int* __restrict__ block_counts) {
  fuse_body<T, D, Q>(VB::hw(), kp, Kk, Df, rec, Ftan, Wtan, lost, nvox, list, count, block_counts);
}

// counters[slot] = sum of n per-block counts (one block, fixed order)
// block-wide integer sum (1-D or 2-D blocks of up to 1024 threads, multiple of 64)
__device__ __forceinline__ int block_sum_int(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __shared__ int ws[16];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  if ((tid & 63) == 0) ws[tid >> 6] = v;
  __syncthreads();
  int s = 0;
  const int nw = int(blockDim.x * blockDim.y) >> 6;
  for (int w = 0; w < nw; ++w) s += ws[w];
  return s;
}
// Per-workgroup counts summed into the frame's counter row (integers: any
// order is exact); advance != nullptr also ends the frame (frame index + 1,
// after every thread has read it).
template <typename T>
__device__ __forceinline__ void sum_counts_body(const VB& vb, const int* __restrict__ a, int n, const int* __restrict__ b, int nb,
                                                              int32_t* __restrict__ counter_base, const int* frame,
                                                              int max_frames, int slot_a, int slot_b, const int* __restrict__ extra,
                                                              int slot_extra, int* advance) {
  int32_t* counters = counter_row(counter_base, frame, max_frames);
  int sa = 0, sb = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) sa += a[i];
  if (b)
    for (int i = threadIdx.x; i < nb; i += blockDim.x) sb += b[i];
  sa = block_sum_int(sa);
  __syncthreads();
  sb = block_sum_int(sb);
  if (threadIdx.x == 0) {
    counters[slot_a] = sa;
    if (b) counters[slot_b] = sb;
    if (extra) counters[slot_extra] = *extra;
    if (advance) *advance += 1;
  }
}
template <typename T>
__global__ __launch_bounds__(1024) void k_sum_counts(const int* __restrict__ a, int n, const int* __restrict__ b, int nb,
                                                     int32_t* __restrict__ counter_base, const int* frame,
                                                     int max_frames, int slot_a, int slot_b, const int* __restrict__ extra,
                                                     int slot_extra, int* advance) {
  sum_counts_body<T>(VB::hw(), a, n, b, nb, counter_base, frame, max_frames, slot_a, slot_b, extra, slot_extra, advance);
}

// Per-brick summary for the raycast: bit 0 = some voxel observed (W > 0),
// bit 1 = every voxel observed with F exactly 1 (free space).  Recomputed for
// the bricks fusion visited (list) or for all bricks (list == nullptr).
// Workgroup 0 also sums the fusion's per-workgroup counts into the frame's
// counter row (fcounts != nullptr): fused voxels and active bricks.
template <typename T>
__device__ __forceinline__ void brick_flags_body(const VB& vb, const typename Vec2<T>::type* __restrict__ rec,
                                                               uint8_t* __restrict__ flags, const int* __restrict__ list,
                                                               const int* __restrict__ count, int nbrick,
                                                               const int* __restrict__ fcounts, int nf,
                                                               int32_t* __restrict__ counter_base,
                                                               const int* __restrict__ frame, int max_frames) {
  if (fcounts && vb.bx == 0) {
    int sf = 0;
    for (int i = threadIdx.x; i < nf; i += blockDim.x) sf += fcounts[i];
    sf = block_sum_int(sf);
    if (threadIdx.x == 0) {
      int32_t* counters = counter_row(counter_base, frame, max_frames);
      counters[1] = sf;
      counters[30] = *count;
    }
  }
  const int nact = list ? *count : nbrick;
  for (int q = vb.bx; q < nact; q += vb.gx) {
    const int b = list ? list[q] : q;
    const auto r = rec[int64_t(b) * kBrickVox + threadIdx.x];
    const int obs = __syncthreads_or(r.y > T(0));
    const int fre = __syncthreads_and(r.y > T(0) && r.x == T(1));
    if (threadIdx.x == 0) flags[b] = uint8_t((obs ? 1 : 0) | (fre ? 2 : 0));
  }
}
template <typename T>
__global__ __launch_bounds__(kBrickVox) void k_brick_flags(const typename Vec2<T>::type* __restrict__ rec,
                                                           uint8_t* __restrict__ flags, const int* __restrict__ list,
                                                           const int* __restrict__ count, int nbrick,
                                                           const int* __restrict__ fcounts, int nf,
                                                           int32_t* __restrict__ counter_base,
                                                           const int* __restrict__ frame, int max_frames) {
  brick_flags_body<T>(VB::hw(), rec, flags, list, count, nbrick, fcounts, nf, counter_base, frame, max_frames);
}

// Bit 2 of a brick's flag: the brick and its seven neighbours in +x, +y, +z
// (the bricks a cell whose lower corner lies in this brick can reach) are all
// free, so every cell with its lower corner here interpolates eight ones.
// Recomputed for every brick after the flags change (a neighbour's update
// changes it); bits 0 and 1, which other threads read here, are not written.
template <typename T>
__device__ __forceinline__ void brick_apron_body(const VB& vb, uint8_t* __restrict__ flags, int nbx, int nby, int nbz) {
  const int b = vb.bx * 256 + threadIdx.x;
  if (b >= nbx * nby * nbz) return;
  const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const uint32_t f = flags[b];
  bool all = (f & 2) && bx + 1 < nbx && by + 1 < nby && bz + 1 < nbz;
  if (all) {
    uint32_t n[7];
#pragma unroll
    for (int c = 1; c < 8; ++c) n[c - 1] = flags[b + (c & 1) + ((c >> 1) & 1) * nbx + (c >> 2) * nbx * nby];
#pragma unroll
    for (int c = 0; c < 7; ++c) all = all && (n[c] & 2);
  }
  flags[b] = uint8_t((f & 3) | (all ? 4 : 0));
}
template <typename T>
__global__ __launch_bounds__(256) void k_brick_apron(uint8_t* __restrict__ flags, int nbx, int nby, int nbz) {
  brick_apron_body<T>(VB::hw(), flags, nbx, nby, nbz);
}

template <typename T, int D, int Q>
__global__ void k_post_track(MPose<D, Q>* Pcur, const MPose<D, Q>* Pinit, KPose<T, D, Q>* Kcur, const int* lost,
                             MPose<D, Q>* history, const int* frame, int max_frames, int* count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  post_track_work(PostTrack<T, D, Q>{Pcur, Pinit, Kcur, lost, history, frame, max_frames, count});
}


// ---------------------------------------------------------------------------
// A7. raycast (Sec. 4.1 "Ray casting", eq. "surface_prediction") and the
// model-map pyramid (level l = level 0 sampled at (2^l x, 2^l y)).
// ---------------------------------------------------------------------------
template <typename T, int D, int Q>
struct MapsOut {
  T* V[3]; T* N[3]; T* Z[3]; uint8_t* valid[3];
};

// trilinear TSDF at a real point given by its grid coordinate g = (v + L/2)/s
// - 1/2 (the caller forms g); valid iff all 8 corners observed (W > 0).
// The brick flags only skip loads: a cell whose first corner lies in a brick
// with no observed voxel is invalid (that corner has W = 0), and a cell inside
// an all-free brick, or with its lower corner in a brick whose +x/+y/+z
// neighbours are all free as well (bit 2), has eight corners equal to 1,
// where the value is taken as 1 without loading them (the march only compares sample values with 0 and
// 0.999, which the interpolation of eight ones meets in the same way).  Brick
// indexes are 32-bit (the brick grid holds far fewer than 2^31 bricks).
template <typename T, int D, int Q>
__device__ __forceinline__ bool trilinear_re(const KParams<T, D, Q>& kp, const typename Vec2<T>::type* __restrict__ rec,
                                             const uint8_t* __restrict__ flags, const T g[3], T& out,
                                             int& cached_brick, uint32_t& cached_flag) {
  int i0[3];
  T f[3];
  bool inb = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T fl = floor(g[a]);
    inb = inb & (fl >= T(0)) & (fl <= T(kp.dim[a] - 2));
    i0[a] = int(fl);
    f[a] = g[a] - fl;
  }
  if (!inb) return false;
  // the flag of the brick holding the lower corner, cached along the ray
  const int bi = ((i0[2] >> 3) * kp.nbr[1] + (i0[1] >> 3)) * kp.nbr[0] + (i0[0] >> 3);
  if (bi != cached_brick) {
    cached_brick = bi;
    cached_flag = flags[bi];
  }
  const uint32_t bf = cached_flag;
  if (!(bf & 1)) return false;
  if ((bf & 4) || ((bf & 2) && (((i0[0] & 7) != 7) & ((i0[1] & 7) != 7) & ((i0[2] & 7) != 7)))) {
    out = T(1);
    return true;
  }
  // all eight records (value and weight) in flight before any is inspected
  typename Vec2<T>::type r[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) r[q] = rec[vox_index(i0[0] + (q & 1), i0[1] + ((q >> 1) & 1), i0[2] + (q >> 2), kp.nbr)];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    pin(r[q].x);
    pin(r[q].y);
  }
  bool ok = true;
  T c[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    ok = ok & (r[q].y > T(0));
    c[q] = r[q].x;
  }
  if (!ok) return false;
  const T fx1 = T(1) - f[0], fy1 = T(1) - f[1], fz1 = T(1) - f[2];
  const T c00 = fx1 * c[0] + f[0] * c[1], c10 = fx1 * c[2] + f[0] * c[3];
  const T c01 = fx1 * c[4] + f[0] * c[5], c11 = fx1 * c[6] + f[0] * c[7];
  const T c0 = fy1 * c00 + f[1] * c10, c1 = fy1 * c01 + f[1] * c11;
  out = fz1 * c0 + f[2] * c1;
  return true;
}

// Complex-step trilinear interpolation, in two steps so that the loads of
// several cells can share one memory round trip: tri_fetch locates the cell of
// a point and issues the loads of its 8 corners (records and tangents; a point
// outside the volume loads a valid cell and is marked invalid), tri_eval checks
// the weights and interpolates.  Valid iff inside and all 8 corners observed.
template <typename T, int D, int Q>
struct TriCell {
  Jet<T, D, Q> f[3];   // fractional position in the cell
  Jet<T, D, Q> c[8];   // corner values with their tangents
  T w[8];              // corner weights
  bool inb;            // inside the volume
};

template <typename T, int D, int Q>
__device__ __forceinline__ void tri_fetch(const KParams<T, D, Q>& kp, const typename Vec2<T>::type* __restrict__ rec,
                                          const T* __restrict__ Ftan, int64_t nvox, const V3<Jet<T, D, Q>>& v,
                                          TriCell<T, D, Q>& t) {
  using J = Jet<T, D, Q>;
  const J* g3[3] = {&v.x, &v.y, &v.z};
  int i0[3];
  t.inb = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const J ga = (*g3[a] + kp.half[a]) / kp.voxel - T(0.5);
    const T fl = floor(ga.re());
    const bool in = fl >= T(0) && fl <= T(kp.dim[a] - 2);
    t.inb = t.inb && in;
    i0[a] = in ? int(fl) : 0;
    t.f[a] = ga - fl;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int64_t id = vox_index(i0[0] + (k & 1), i0[1] + ((k >> 1) & 1), i0[2] + (k >> 2), kp.nbr);
    const auto r = rec[id];
    t.w[k] = r.y;
    t.c[k].v[0] = r.x;
#pragma unroll
    for (int q = 1; q < J::N; ++q) t.c[k].v[q] = Ftan[size_t(q - 1) * nvox + id];
  }
}

// keeps the loads of a fetched cell ahead of the next branch (few components
// only: many components would hold too many registers in flight)
template <typename T, int D, int Q>
__device__ __forceinline__ void tri_pin(TriCell<T, D, Q>& t) {
  if constexpr (Jet<T, D, Q>::N <= 4) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      pin(t.w[k]);
      pin(t.c[k]);
    }
  }
}

template <typename T, int D, int Q>
__device__ __forceinline__ bool tri_eval(const TriCell<T, D, Q>& t, Jet<T, D, Q>& out) {
  using J = Jet<T, D, Q>;
  bool ok = t.inb;
#pragma unroll
  for (int k = 0; k < 8; ++k) ok = ok & (t.w[k] > T(0));
  if (!ok) return false;
  const J* c = t.c;
  const J one = jconst<J>(T(1));
  const J fx1 = one - t.f[0], fy1 = one - t.f[1], fz1 = one - t.f[2];
  const J c00 = fx1 * c[0] + t.f[0] * c[1], c10 = fx1 * c[2] + t.f[0] * c[3];
  const J c01 = fx1 * c[4] + t.f[0] * c[5], c11 = fx1 * c[6] + t.f[0] * c[7];
  const J c0 = fy1 * c00 + t.f[1] * c10, c1 = fy1 * c01 + t.f[1] * c11;
  out = fz1 * c0 + t.f[2] * c1;
  return true;
}

// The ray o + alpha R K^-1 (u,1) is marched on real parts only: half a voxel
// while the last sample is observed and inside the band (F < 0.999), else
// 0.8 mu; from max(near, entry) to the exit of the volume shrunk by one voxel.
// F_m > 0 > F_{m+1} between consecutive valid samples is a hit; - to + stops
// the ray.  This kernel records, per pixel, the bracketing alphas of the hit
// (a negative second alpha: no hit); k_rayhit evaluates it in complex-step
// arithmetic.  Real parts here are computed with the same operations as the
// real parts of k_rayhit's jets.
template <typename T, int D, int Q>
__device__ __forceinline__ void raymarch_body(const VB& vb, const KParams<T, D, Q>& kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                            const typename Vec2<T>::type* __restrict__ rec,
                                                            const uint8_t* __restrict__ flags,
                                                            typename Vec2<T>::type* __restrict__ bracket,
                                                            int* __restrict__ block_samples) {
  const int tile = xcd_remap(vb.by * vb.gx + vb.bx, vb.gx * vb.gy);
  const int x = (tile % vb.gx) * blockDim.x + threadIdx.x, y = (tile / vb.gx) * blockDim.y + threadIdx.y;
  const int W = kp.W, H = kp.H;
  int nsamp = 0;
  if (x < W && y < H) {
    using R0 = Jet<T, 0, 0>;
    const KPose<T, D, Q>& P = *Kk;
    KPose<T, 0, 0> Pr;
#pragma unroll
    for (int q = 0; q < 9; ++q) Pr.R[q].v[0] = P.R[q].re();
#pragma unroll
    for (int q = 0; q < 3; ++q) Pr.t[q].v[0] = P.t[q].re();
    const V3<R0> dh = {(jconst<R0>(T(x)) - kp.cx.re()) / jconst<R0>(kp.fx.re()),
                       (jconst<R0>(T(y)) - kp.cy.re()) / jconst<R0>(kp.fy.re()), jconst<R0>(T(1))};
    const V3<R0> dir = pose_rotate(Pr, dh);
    const T orr[3] = {Pr.t[0].re(), Pr.t[1].re(), Pr.t[2].re()};
    const T dr[3] = {dir.x.re(), dir.y.re(), dir.z.re()};
    const T nrm = sqrt(dh.x.re() * dh.x.re() + dh.y.re() * dh.y.re() + T(1));
    const T s = kp.voxel;
    T tmin = T(-1e30), tmax = T(1e30);
    bool miss = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T lo = -kp.half[a] + s, hi = kp.half[a] - s;
      if (dr[a] != T(0)) {
        const T t1 = (lo - orr[a]) / dr[a], t2 = (hi - orr[a]) / dr[a];
        tmin = fmax(tmin, fmin(t1, t2));
        tmax = fmin(tmax, fmax(t1, t2));
      } else if (orr[a] < lo || orr[a] > hi) {
        miss = true;
      }
    }
    // the ray parameter accumulates over up to hundreds of samples: FP32 runs
    // keep it (and the sample coordinates) in FP64, so that the sample grid
    // does not drift by the rounding of every step
    using TA = typename std::conditional<std::is_same<T, float>::value, double, T>::type;
    TA alpha = fmax(TA(kp.near_m), TA(tmin));
    const T mu = kp.mu.re();
    TA small = TA(0.5) * TA(s) / TA(nrm), big = TA(0.8) * TA(mu) / TA(nrm);
    // (opaque from here: otherwise the compiler folds the two divisions into
    // one of the selected numerator, inside the loop)
    pin(small);
    pin(big);
    bool prev_ok = false;
    TA a_prev = 0;
    T f_prev = 0;
    TA hit0 = 0, hit1 = TA(-1);
    int cbrick = -1;
    uint32_t cflag = 0;
    // FP32 runs: the grid coordinate of the sample is G0 + alpha dG, formed
    // in FP64 (one fma per axis) and rounded once; FP64 runs evaluate
    // ((o + alpha d) + L/2) / s - 1/2 as written
    TA G0[3], dG[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      G0[a] = (TA(orr[a]) + TA(kp.half[a])) / TA(kp.voxel) - TA(0.5);
      dG[a] = TA(dr[a]) / TA(kp.voxel);
    }
    for (int it = 0; it < 100000 && !miss && alpha <= TA(tmax); ++it, ++nsamp) {
      T g[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if constexpr (std::is_same<T, float>::value) g[a] = T(fma(alpha, dG[a], G0[a]));
        else g[a] = ((orr[a] + alpha * dr[a]) + kp.half[a]) / kp.voxel - T(0.5);
      }
      T f;
      const bool okf = trilinear_re(kp, rec, flags, g, f, cbrick, cflag);
      if (!okf) f = 0;
      if (okf && prev_ok) {
        if (f_prev > T(0) && f < T(0)) {
          hit0 = a_prev;
          hit1 = alpha;
          break;
        }
        if (f_prev < T(0) && f > T(0)) break;
      }
      const TA step = (okf && f < T(0.999)) ? small : big;
      prev_ok = okf;
      a_prev = alpha;
      f_prev = f;
      alpha = alpha + step;
    }
    typename Vec2<T>::type b;
    b.x = T(hit0);
    b.y = T(hit1);
    bracket[size_t(y) * W + x] = b;
  }
  const int ns = block_sum_int(nsamp);
  if (threadIdx.x == 0 && threadIdx.y == 0) block_samples[vb.by * vb.gx + vb.bx] = ns;
}
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_raymarch(KParams<T, D, Q> kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                  const typename Vec2<T>::type* __restrict__ rec,
                                                  const uint8_t* __restrict__ flags,
                                                  typename Vec2<T>::type* __restrict__ bracket,
                                                  int* __restrict__ block_samples) {
  raymarch_body<T, D, Q>(VB::hw(), kp, Kk, rec, flags, bracket, block_samples);
}

// Complex-step evaluation of a bracketed crossing: alpha0 = alpha_m -
// dalpha F_m / (F_{m+1} - F_m) (eq. after the crossing test), V = r(alpha0),
// N = normalised central difference of F at +-1 voxel; writes the model maps
// of levels 0-2.
template <typename T, int D, int Q>
__device__ __forceinline__ void rayhit_body(const VB& vb, const KParams<T, D, Q>& kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                          const typename Vec2<T>::type* __restrict__ rec,
                                                          const T* __restrict__ Ftan, int64_t nvox,
                                                          const typename Vec2<T>::type* __restrict__ bracket,
                                                          const MapsOut<T, D, Q>& out, int* __restrict__ block_hits) {
  using J = Jet<T, D, Q>;
  const int tile = xcd_remap(vb.by * vb.gx + vb.bx, vb.gx * vb.gy);
  const int x = (tile % vb.gx) * blockDim.x + threadIdx.x, y = (tile / vb.gx) * blockDim.y + threadIdx.y;
  const int W = kp.W, H = kp.H;
  const bool inside = x < W && y < H;
  bool ok = false;
  const J z = jzero<J>();
  V3<J> Vg = {z, z, z}, Ng = {z, z, z};
  T zhit = 0;
  if (inside) {
    const auto br = bracket[size_t(y) * W + x];
    if (br.y >= T(0)) {
      const T a_prev = br.x, alpha = br.y;
      const KPose<T, D, Q>& P = *Kk;
      const V3<J> dh = {(jconst<J>(T(x)) - kp.cx) / kp.fx, (jconst<J>(T(y)) - kp.cy) / kp.fy, jconst<J>(T(1))};
      const V3<J> dir = pose_rotate(P, dh);
      const V3<J> o = {P.t[0], P.t[1], P.t[2]};
      const T s = kp.voxel;
      J F0, F1;
      const V3<J> v0 = vadd(o, vscale(jconst<J>(a_prev), dir));
      const V3<J> v1 = vadd(o, vscale(jconst<J>(alpha), dir));
      bool ok01;
      {
        TriCell<T, D, Q> t0, t1;
        tri_fetch(kp, rec, Ftan, nvox, v0, t0);
        tri_fetch(kp, rec, Ftan, nvox, v1, t1);
        tri_pin(t0);
        tri_pin(t1);
        const bool ok0 = tri_eval(t0, F0);
        const bool ok1 = tri_eval(t1, F1);
        ok01 = ok0 && ok1;
      }
      if (ok01) {
        const J a0 = jconst<J>(a_prev) - jconst<J>(alpha - a_prev) * F0 / (F1 - F0);
        const V3<J> V = vadd(o, vscale(a0, dir));
        J gr[3];
        bool okg = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          V3<J> vp = V, vm = V;
          if (a == 0) { vp.x = V.x + s; vm.x = V.x - s; }
          if (a == 1) { vp.y = V.y + s; vm.y = V.y - s; }
          if (a == 2) { vp.z = V.z + s; vm.z = V.z - s; }
          // the two cells of one axis in flight together
          TriCell<T, D, Q> tp, tm;
          tri_fetch(kp, rec, Ftan, nvox, vp, tp);
          tri_fetch(kp, rec, Ftan, nvox, vm, tm);
          tri_pin(tp);
          tri_pin(tm);
          J fp, fm;
          const bool okp = tri_eval(tp, fp);
          const bool okm = tri_eval(tm, fm);
          okg = okg && okp && okm;
          if (okg) gr[a] = fp - fm;
        }
        if (okg) {
          const V3<J> gv = {gr[0], gr[1], gr[2]};
          const J gg = vdot(gv, gv);
          if (gg.re() > T(0)) {
            ok = true;
            Vg = V;
            Ng = vscale(jconst<J>(T(1)) / jsqrt(gg), gv);
            zhit = a0.re();
          }
        }
      }
    }
  }
  const int nh = block_sum_int(ok ? 1 : 0);
  if (threadIdx.x == 0 && threadIdx.y == 0) block_hits[vb.by * vb.gx + vb.bx] = nh;
  if (!inside) return;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if ((x & ((1 << l) - 1)) || (y & ((1 << l) - 1))) break;
    const int Wl = W >> l, Hl = H >> l;
    const size_t nl = size_t(Wl) * Hl, il = size_t(y >> l) * Wl + (x >> l);
    vstore(out.V[l], nl, il, Vg);
    vstore(out.N[l], nl, il, Ng);
    out.Z[l][il] = zhit;
    out.valid[l][il] = ok ? 1 : 0;
  }
}
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_rayhit(KParams<T, D, Q> kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                const typename Vec2<T>::type* __restrict__ rec,
                                                const T* __restrict__ Ftan, int64_t nvox,
                                                const typename Vec2<T>::type* __restrict__ bracket,
                                                MapsOut<T, D, Q> out, int* __restrict__ block_hits) {
  rayhit_body<T, D, Q>(VB::hw(), kp, Kk, rec, Ftan, nvox, bracket, out, block_hits);
}

// ---------------------------------------------------------------------------
// learned initialiser plumbing
// ---------------------------------------------------------------------------
// Network input parts at pyramid level 3 (80 x 60 for 640 x 480): the depth
// channel is the level-2 filtered depth reduced once more with the pyramid's
// gated binomial (real parts); the model channels are the level-0 model maps
// sampled at (8x, 8y): hit depth and the normal rotated into the camera frame
// of pose Km.  Invalid pixels are 0.
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_cnn_parts(KParams<T, D, Q> kp, const T* __restrict__ D2,
                                                   const T* __restrict__ Nm0, const T* __restrict__ Zm0,
                                                   const uint8_t* __restrict__ mvalid0,
                                                   const KPose<T, D, Q>* __restrict__ Km, float* __restrict__ out_depth,
                                                   float* __restrict__ out_model) {
  constexpr int NC = Jet<T, D, Q>::N;
  const int W3 = kp.W >> 3, H3 = kp.H >> 3, W2 = kp.W >> 2, H2 = kp.H >> 2;
  const int x = blockIdx.x * 16 + threadIdx.x, y = blockIdx.y * 16 + threadIdx.y;
  if (x >= W3 || y >= H3) return;
  const int o = y * W3 + x;
  // depth, level 3
  float dv = 0.f;
  const T c = D2[size_t(2 * y) * W2 + 2 * x];
  if (c > T(0)) {
    const int g[5] = {1, 4, 6, 4, 1};
    T num = 0, den = 0;
    for (int j = -2; j <= 2; ++j)
      for (int i = -2; i <= 2; ++i) {
        const int xx = 2 * x + i, yy = 2 * y + j;
        if (xx < 0 || yy < 0 || xx >= W2 || yy >= H2) continue;
        const T d = D2[size_t(yy) * W2 + xx];
        if (!(d > T(0)) || fabs(d - c) > kp.pyr_gate) continue;
        const T w = T(g[i + 2] * g[j + 2]);
        num += w * d;
        den += w;
      }
    dv = float(num / den);
  }
  out_depth[o] = dv;
  // model, level 0 at (8x, 8y)
  const size_t n0 = size_t(kp.W) * kp.H, s0 = size_t(8 * y) * kp.W + 8 * x;
  float z = 0.f, nx = 0.f, ny = 0.f, nz = 0.f;
  if (mvalid0[s0]) {
    const T wx = Nm0[0 * NC * n0 + s0], wy = Nm0[1 * NC * n0 + s0], wz = Nm0[2 * NC * n0 + s0];
    const KPose<T, D, Q>& P = *Km;
    z = float(Zm0[s0]);
    nx = float(P.R[0].re() * wx + P.R[3].re() * wy + P.R[6].re() * wz);
    ny = float(P.R[1].re() * wx + P.R[4].re() * wy + P.R[7].re() * wz);
    nz = float(P.R[2].re() * wx + P.R[5].re() * wy + P.R[8].re() * wz);
  }
  const int n3 = W3 * H3;
  out_model[o] = z;
  out_model[n3 + o] = nx;
  out_model[2 * n3 + o] = ny;
  out_model[3 * n3 + o] = nz;
}

// the two initial-pose candidates: network T_{k-1} exp(xi) (real increment,
// the tangents come from T_{k-1}) and the previous / constant-velocity pose
// already in Pinit; the network candidate becomes the current estimate
template <typename T, int D, int Q>
__global__ void k_init_candidates(const MPose<D, Q>* Pprev, const MPose<D, Q>* Pinit, const float* xi,
                                  MPose<D, Q>* Pcand, MPose<D, Q>* Pcur, KPose<T, D, Q>* Kcur) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  using JD = Jet<double, D, Q>;
  JD d[6];
  for (int a = 0; a < 6; ++a) d[a] = jconst<JD>(double(xi[a]));
  const MPose<D, Q> Tn = pose_mul(*Pprev, se3_exp<D, Q>(d));
  *Pcand = Tn;
  *Pcur = Tn;
  *Kcur = to_kpose<T, double>(Tn);
  (void)Pinit;
}

template <typename T, int D, int Q>
__global__ void k_set_current(const MPose<D, Q>* P, MPose<D, Q>* Pcur, KPose<T, D, Q>* Kcur) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  *Pcur = *P;
  *Kcur = to_kpose<T, double>(*P);
}

// keep the candidate with the lower mean squared residual of one level-2 pass;
// the network's only with at least 100 correspondences and at least 95% of
// the constant-velocity candidate's (a candidate that loses correspondences
// to the gates can show a lower mean residual while being further off)
template <typename T, int D, int Q>
__global__ void k_choose_init(const double* sums_net, const double* sums_cv, int ns, const MPose<D, Q>* Pnet,
                              MPose<D, Q>* Pinit, MPose<D, Q>* Pcur, KPose<T, D, Q>* Kcur, int32_t* counter_base,
                              const int* frame, int max_frames) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t* crow = counter_row(counter_base, frame, max_frames);
  const double cn = sums_net[ns - 2], cc = sums_cv[ns - 2];
  const double en = cn > 0 ? sums_net[ns - 1] / cn : 1e300, ec = cc > 0 ? sums_cv[ns - 1] / cc : 1e300;
  const bool use_net = cn >= 100.0 && cn >= 0.95 * cc && en < ec;
  if (use_net) *Pinit = *Pnet;
  *Pcur = *Pinit;
  *Kcur = to_kpose<T, double>(*Pinit);
  crow[33] = use_net ? 1 : 0;
}

// ---------------------------------------------------------------------------
// trajectory error (translational RMSE, no alignment), FP64
// ---------------------------------------------------------------------------
template <int D, int Q>
__global__ void k_traj_err(const MPose<D, Q>* hist, const double* gt, int n, double* out) {
  using J = Jet<double, D, Q>;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  J acc = jzero<J>();
  double ss[D > 0 ? D : 1] = {};
  for (int k = 0; k < n; ++k)
    for (int r = 0; r < 3; ++r) {
      J d = hist[k].m[9 + r] - gt[k * 16 + r * 4 + 3];
      acc = acc + d * d;
      for (int a = 0; a < D; ++a) ss[a] = fma(d.v[1 + a], d.v[1 + a], ss[a]);
    }
  if (acc.v[0] == 0.0) {
    // the trajectory equals the reference: E = |d|/sqrt(n) has a kink at d = 0
    // and sqrt's derivative is unbounded there.  The derivative along +theta_a
    // is the one-sided |d_a|/sqrt(n) (what full complex arithmetic gives:
    // sqrt(-sum d_a^2 / n) = i |d_a|/sqrt(n)); second-order parts are 0.
    out[0] = 0.0;
    for (int a = 0; a < D; ++a) out[1 + a] = sqrt(ss[a] / double(n));
    for (int c = 1 + D; c < J::N; ++c) out[c] = 0.0;
    return;
  }
  J e = jsqrt(acc / double(n));
  for (int c = 0; c < J::N; ++c) out[c] = e.v[c];
}

// ---------------------------------------------------------------------------
// layout conversion between bricks and x-fastest linear order (get/set)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_vol_gather(const typename Vec2<T>::type* rec, const T* Ftan, const T* Wtan, int comp_kind,
                             int comp, int64_t nvox, int nx, int ny, int nbx, int nby, int64_t start, int64_t count,
                             T* dst) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= count) return;
  int64_t li = start + q;
  int i = int(li % nx), j = int((li / nx) % ny), k = int(li / (int64_t(nx) * ny));
  int nbr[3] = {nbx, nby, 0};
  int64_t vi = vox_index(i, j, k, nbr);
  T v;
  if (comp_kind == 0) v = rec[vi].x;                       // F real
  else if (comp_kind == 1) v = rec[vi].y;                  // W real
  else if (comp_kind == 2) v = Ftan[size_t(comp) * nvox + vi];
  else v = Wtan ? Wtan[vi] : T(0);                         // W weight-cap part
  dst[q] = v;
}

template <typename T>
__global__ void k_vol_scatter(typename Vec2<T>::type* rec, T* Ftan, T* Wtan, int comp_kind, int comp, int64_t nvox,
                              int nx, int ny, int nbx, int nby, int64_t start, int64_t count, const T* src) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= count) return;
  int64_t li = start + q;
  int i = int(li % nx), j = int((li / nx) % ny), k = int(li / (int64_t(nx) * ny));
  int nbr[3] = {nbx, nby, 0};
  int64_t vi = vox_index(i, j, k, nbr);
  T v = src[q];
  if (comp_kind == 0) rec[vi].x = v;
  else if (comp_kind == 1) rec[vi].y = v;
  else if (comp_kind == 2) Ftan[size_t(comp) * nvox + vi] = v;
  else if (Wtan) Wtan[vi] = v;
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

}  // namespace xs
