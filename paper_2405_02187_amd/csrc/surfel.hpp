// X-PointFusion front end (Sec. 4.2): a surfel map in place of the TSDF.
//
// Global model points (surfels) carry a position v, a normal n, a radius r, a
// confidence c and a time stamp t; v, n, r, c are jets, so they carry the
// perturbation's parts exactly as the TSDF does.  Per frame, after tracking:
//
//  1. the surfels are rendered at the tracked pose into an index map at 4 x 4
//     the image resolution (k_surf_project: one 64-bit key per sub-pixel, the
//     camera depth rounded to FP32 in the high word and the surfel index in the
//     low word, kept by atomicMin: the nearest surfel, ties to the lower index,
//     whatever the order of the atomics);
//  2. every valid measured pixel takes the surfels of its 4 x 4 block that
//     pass the depth-along-ray, normal-angle and distance gates (decided on
//     real parts) and updates all of them (one-to-many) with the Gaussian
//     weight of their distance to the measured point times the measurement's
//     confidence exp(-gamma^2 / 0.72) (k_surf_assoc).  Each surfel lies in one
//     sub-pixel, so each is written by at most one thread;
//  3. pixels with no qualified surfel become new surfels, appended in pixel
//     order through a two-level prefix sum (k_surf_count, k_surf_scan,
//     k_surf_insert), up to the capacity;
//  4. the model maps for the next frame's ICP are the nearest surfel per pixel
//     (an index map at 1 x over the surfels whose confidence reaches c_stable)
//     with its position, unit normal and camera depth, levels 1-2 by
//     subsampling (k_surf_project, k_surf_maps).
//
// Surfel arrays, capacity `cap`: v, n [3][NC][cap], r, c [NC][cap], t [cap].
#pragma once
#include "kernels.hpp"

namespace xs {

constexpr unsigned long long kSurfEmpty = ~0ull;
constexpr int kSurfScanBlock = 1024;     // pixels per block of the insertion prefix sum

struct SurfCfg {
  double d_depth;     // |camera z of the surfel - measured z| gate (m)
  double cos_norm;    // cosine of the normal-angle gate
  double d_dist;      // distance gate to the measured point (m)
  double two_s2;      // 2 sigma^2 of the Gaussian weight (m^2)
  double c_stable;    // confidence floor of the predicted model maps
  int cap;            // capacity
};

template <typename T>
struct SurfMap {
  T* v; T* n; T* r; T* c;
  int32_t* t;
  int* count;         // surfels in use
  int* base;          // count before this frame's insertions
};

// real position of surfel i (plane 0 of each axis)
template <typename T, int NC>
__device__ __forceinline__ void surf_pos_re(const SurfMap<T>& m, int cap, int i, T p[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) p[a] = m.v[size_t(a * NC) * cap + i];
}

// camera-frame z and image position of a real world point under the real pose
template <typename T, int D, int Q>
__device__ __forceinline__ bool surf_project(const KParams<T, D, Q>& kp, const KPose<T, D, Q>& P, const T p[3], T& z,
                                             T& ux, T& uy) {
  const T d0 = p[0] - P.t[0].re(), d1 = p[1] - P.t[1].re(), d2 = p[2] - P.t[2].re();
  const T x = P.R[0].re() * d0 + P.R[3].re() * d1 + P.R[6].re() * d2;
  const T y = P.R[1].re() * d0 + P.R[4].re() * d1 + P.R[7].re() * d2;
  z = P.R[2].re() * d0 + P.R[5].re() * d1 + P.R[8].re() * d2;
  if (!(z > T(0))) return false;
  ux = kp.fx.re() * x / z + kp.cx.re();
  uy = kp.fy.re() * y / z + kp.cy.re();
  return true;
}

// index map at `sup` x the image: the nearest surfel per sub-pixel among those
// with confidence >= c_min (the map starts filled with kSurfEmpty)
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_surf_project(KParams<T, D, Q> kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                      SurfMap<T> m, int cap, int sup, double c_min,
                                                      unsigned long long* __restrict__ map) {
  constexpr int NC = Jet<T, D, Q>::N;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= *m.count) return;
  if (!(double(m.c[i]) >= c_min)) return;
  const KPose<T, D, Q>& P = *Kk;
  T p[3], z, ux, uy;
  surf_pos_re<T, NC>(m, cap, i, p);
  if (!surf_project(kp, P, p, z, ux, uy)) return;
  const T ax = floor(T(sup) * (ux + T(0.5))), ay = floor(T(sup) * (uy + T(0.5)));
  const int WS = kp.W * sup, HS = kp.H * sup;
  if (!(ax >= T(0) && ay >= T(0) && ax < T(WS) && ay < T(HS))) return;
  const unsigned long long key =
      (static_cast<unsigned long long>(__float_as_uint(float(z))) << 32) | static_cast<unsigned>(i);
  atomicMin(&map[size_t(ay) * WS + size_t(ax)], key);
}

// measurement confidence exp(-gamma^2 / 0.72), gamma the radial distance of
// pixel (x, y) from the principal point over that of the image corner
template <typename T, int D, int Q>
__device__ __forceinline__ Jet<T, D, Q> surf_confidence(const KParams<T, D, Q>& kp, int x, int y) {
  using J = Jet<T, D, Q>;
  const J dx = jconst<J>(T(x)) - kp.cx, dy = jconst<J>(T(y)) - kp.cy;
  const J g2 = (dx * dx + dy * dy) / (kp.cx * kp.cx + kp.cy * kp.cy);
  return jexp(-g2 / T(0.72));
}

// surfel radius of a measurement: sqrt(2) z / (f |n_z|), |n_z| >= 0.25
template <typename T, int D, int Q>
__device__ __forceinline__ Jet<T, D, Q> surf_radius(const KParams<T, D, Q>& kp, const V3<Jet<T, D, Q>>& Vc,
                                                    const V3<Jet<T, D, Q>>& Nc) {
  using J = Jet<T, D, Q>;
  J nz = Nc.z.re() < T(0) ? -Nc.z : Nc.z;
  if (nz.re() < T(0.25)) nz = jconst<J>(T(0.25));
  return T(1.4142135623730951) * Vc.z / (kp.fx * nz);
}

// association and one-to-many update; fresh[u] = 1 for a valid pixel with no
// qualified surfel (a new surfel); per-workgroup update counts
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_surf_assoc(KParams<T, D, Q> kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                    const T* __restrict__ Vl0, const T* __restrict__ Nl0,
                                                    const uint8_t* __restrict__ valid0, SurfMap<T> m, SurfCfg sc,
                                                    const unsigned long long* __restrict__ map4,
                                                    uint8_t* __restrict__ fresh, const int* __restrict__ lost,
                                                    const int* __restrict__ frame, int* __restrict__ block_upd) {
  using J = Jet<T, D, Q>;
  constexpr int NC = J::N;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
  const int W = kp.W, H = kp.H;
  const bool inside = x < W && y < H;
  const size_t n = size_t(W) * H, u = size_t(y) * W + x;
  int upd = 0;
  bool isnew = false;
  if (inside && !*lost && valid0[u]) {
    const KPose<T, D, Q>& P = *Kk;
    const int cap = sc.cap, k = *frame;
    const V3<J> Vc = vload<J>(Vl0, n, u), Nc = vload<J>(Nl0, n, u);
    const V3<J> Vg = pose_apply(P, Vc), Ng = pose_rotate(P, Nc);
    const T vg[3] = {Vg.x.re(), Vg.y.re(), Vg.z.re()}, ng[3] = {Ng.x.re(), Ng.y.re(), Ng.z.re()};
    const T zu = Vc.z.re();
    const J Cu = surf_confidence(kp, x, y);
    const J rnew = surf_radius(kp, Vc, Nc);
    for (int sy = 0; sy < 4; ++sy)
      for (int sx = 0; sx < 4; ++sx) {
        const unsigned long long key = map4[size_t(4 * y + sy) * (4 * W) + size_t(4 * x + sx)];
        if (key == kSurfEmpty) continue;
        const int i = int(unsigned(key & 0xffffffffull));
        // gates on real parts
        T p[3], zi, ux, uy;
        surf_pos_re<T, NC>(m, cap, i, p);
        surf_project(kp, P, p, zi, ux, uy);
        if (!(fabs(zi - zu) <= T(sc.d_depth))) continue;
        const T n0 = m.n[size_t(0 * NC) * cap + i], n1 = m.n[size_t(1 * NC) * cap + i],
                n2 = m.n[size_t(2 * NC) * cap + i];
        const T nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        if (!(nn > T(0)) || !(n0 * ng[0] + n1 * ng[1] + n2 * ng[2] >= T(sc.cos_norm) * nn)) continue;
        const T e0 = p[0] - vg[0], e1 = p[1] - vg[1], e2 = p[2] - vg[2];
        if (!(sqrt(e0 * e0 + e1 * e1 + e2 * e2) <= T(sc.d_dist))) continue;
        // the update with the Gaussian weight of the distance
        const V3<J> vi = vload<J>(m.v, cap, i), ni = vload<J>(m.n, cap, i);
        const J ri = jload<J>(m.r, cap, i), ci = jload<J>(m.c, cap, i);
        const V3<J> d = vsub(vi, Vg);
        const J w = jexp(-vdot(d, d) / T(sc.two_s2));
        const J a = w * Cu;
        const J den = ci + a;
        const J inv = jconst<J>(T(1)) / den;
        vstore(m.v, cap, i, vscale(inv, vadd(vscale(ci, vi), vscale(a, Vg))));
        vstore(m.n, cap, i, vscale(inv, vadd(vscale(ci, ni), vscale(a, Ng))));
        jstore(m.r, cap, i, (ci * ri + a * rnew) / den);
        jstore(m.c, cap, i, den);
        m.t[i] = k;
        ++upd;
      }
    isnew = upd == 0;
  }
  if (inside) fresh[u] = isnew ? 1 : 0;
  const int s = block_sum_int(upd);
  if (threadIdx.x == 0 && threadIdx.y == 0) block_upd[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// new surfels per block of kSurfScanBlock pixels (T: the context precision;
// one instance per shape)
template <typename T>
__global__ __launch_bounds__(kSurfScanBlock) void k_surf_count(const uint8_t* __restrict__ fresh, int npx,
                                                               int* __restrict__ bcnt) {
  const int u = blockIdx.x * kSurfScanBlock + threadIdx.x;
  const int s = block_sum_int(u < npx && fresh[u] ? 1 : 0);
  if (threadIdx.x == 0) bcnt[blockIdx.x] = s;
}

// exclusive prefix over the blocks (one workgroup, fixed order), the frame's
// insertion count within the capacity, the update count; counters: 1 surfel
// updates, 35 inserted, 36 dropped at the capacity, 37 surfels in use
template <typename T>
__global__ __launch_bounds__(1024) void k_surf_scan(const int* __restrict__ bcnt, int nblk, int* __restrict__ boff,
                                                    const int* __restrict__ block_upd, int nupd, int* count, int* base,
                                                    int cap, int32_t* __restrict__ counter_base,
                                                    const int* __restrict__ frame, int max_frames) {
  __shared__ int wtot[16];
  int upd = 0;
  for (int i = threadIdx.x; i < nupd; i += blockDim.x) upd += block_upd[i];
  upd = block_sum_int(upd);
  // serial chunks of the block counts, one per thread, then an exclusive scan
  // of the chunk sums (wave scans, then the scan of the 16 wave totals)
  const int per = (nblk + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  int s = 0;
  for (int b = b0; b < b0 + per && b < nblk; ++b) s += bcnt[b];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(inc, o, 64);
    if (lane >= o) inc += v;
  }
  if (lane == 63) wtot[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < 16; ++w) {
      const int v = wtot[w];
      wtot[w] = acc;
      acc += v;
    }
    const int c0 = *count;
    const int ins = min(acc, cap - c0);
    *base = c0;
    *count = c0 + ins;
    int32_t* row = counter_row(counter_base, frame, max_frames);
    row[1] = upd;
    row[35] = ins;
    row[36] = acc - ins;
    row[37] = c0 + ins;
  }
  __syncthreads();
  int acc = wtot[wv] + inc - s;
  for (int b = b0; b < b0 + per && b < nblk; ++b) {
    boff[b] = acc;
    acc += bcnt[b];
  }
}

// the new surfels, in pixel order (block offset + rank within the block)
template <typename T, int D, int Q>
__global__ __launch_bounds__(kSurfScanBlock) void k_surf_insert(KParams<T, D, Q> kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                                const T* __restrict__ Vl0, const T* __restrict__ Nl0,
                                                                const uint8_t* __restrict__ fresh,
                                                                const int* __restrict__ boff, SurfMap<T> m, int cap,
                                                                const int* __restrict__ frame) {
  using J = Jet<T, D, Q>;
  constexpr int NW = kSurfScanBlock / 64;
  __shared__ int wc[NW];
  const int W = kp.W, H = kp.H;
  const int npx = W * H;
  const int u = blockIdx.x * kSurfScanBlock + threadIdx.x;
  const bool f = u < npx && fresh[u];
  const unsigned long long bal = __ballot(f);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) wc[wv] = int(__popcll(bal));
  __syncthreads();
  if (!f) return;
  int rank = boff[blockIdx.x];
  for (int w = 0; w < wv; ++w) rank += wc[w];
  rank += int(__popcll(bal & ((1ull << lane) - 1ull)));
  const int pos = *m.base + rank;
  if (pos >= *m.count) return;                 // beyond the capacity: dropped
  const KPose<T, D, Q>& P = *Kk;
  const size_t n = size_t(npx);
  const int x = u % W, y = u / W;
  const V3<J> Vc = vload<J>(Vl0, n, u), Nc = vload<J>(Nl0, n, u);
  vstore(m.v, cap, pos, pose_apply(P, Vc));
  vstore(m.n, cap, pos, pose_rotate(P, Nc));
  jstore(m.r, cap, pos, surf_radius(kp, Vc, Nc));
  jstore(m.c, cap, pos, surf_confidence(kp, x, y));
  m.t[pos] = *frame;
  (void)H;
}

// model maps of levels 0-2 from the 1x index map: position, unit normal,
// camera depth of the nearest stable surfel; per-workgroup hit counts
template <typename T, int D, int Q>
__global__ __launch_bounds__(256) void k_surf_maps(KParams<T, D, Q> kp, const KPose<T, D, Q>* __restrict__ Kk,
                                                   SurfMap<T> m, int cap,
                                                   const unsigned long long* __restrict__ map1, MapsOut<T, D, Q> out,
                                                   int* __restrict__ block_hits) {
  using J = Jet<T, D, Q>;
  constexpr int NC = J::N;
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
  const int W = kp.W, H = kp.H;
  const bool inside = x < W && y < H;
  const J z0 = jzero<J>();
  V3<J> Vg = {z0, z0, z0}, Ng = {z0, z0, z0};
  T zhit = 0;
  bool ok = false;
  if (inside) {
    const unsigned long long key = map1[size_t(y) * W + x];
    if (key != kSurfEmpty) {
      const int i = int(unsigned(key & 0xffffffffull));
      const V3<J> ni = vload<J>(m.n, cap, i);
      const J nn = jsqrt(vdot(ni, ni));
      if (nn.re() > T(0)) {
        ok = true;
        Vg = vload<J>(m.v, cap, i);
        Ng = vscale(jconst<J>(T(1)) / nn, ni);
        T p[3], ux, uy;
        surf_pos_re<T, NC>(m, cap, i, p);
        surf_project(kp, *Kk, p, zhit, ux, uy);
      }
    }
  }
  const int nh = block_sum_int(ok ? 1 : 0);
  if (threadIdx.x == 0 && threadIdx.y == 0) block_hits[blockIdx.y * gridDim.x + blockIdx.x] = nh;
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

}  // namespace xs
