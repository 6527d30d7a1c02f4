// Orchestration of the frame step for one (precision, directions, Hessian) shape.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <cmath>
#include <functional>
#include <string>
#include <type_traits>
#include <vector>
#include "ctx.hpp"
#include "kernels.hpp"
#include "newton.hpp"
#include "reloc.hpp"
#include "surfel.hpp"
#include "group.hpp"

namespace xs {

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// sub-allocation of the caller's workspace
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(char* b) : base(b) {}
  template <typename P> P* take(size_t count) {
    size_t o = off;
    off = align_up(off + count * sizeof(P));
    return base ? reinterpret_cast<P*>(base + o) : nullptr;
  }
};

template <typename T, int D, int Q>
struct Engine : EngineBase {
  using J = Jet<T, D, Q>;
  using JD = Jet<double, D, Q>;
  using T2 = typename Vec2<T>::type;
  static constexpr int NC = J::N;
  static constexpr int NS = IcpSize<D, Q>::NS;
  static constexpr int64_t kStageElems = int64_t(1) << 22;
  static constexpr int kFuseBlocks = 4096;

  xslam_ctx_s* C;
  KParams<T, D, Q> kp;
  JD omega[3];
  int W[3], H[3];
  size_t npx[3];
  int64_t nvox = 0;
  int nbrick = 0;
  int ndepth = 0;       // depth_dot planes
  int frame = 0;        // host mirror of the processed-frame count
  bool measured = false, have_model = false;

  // device buffers
  T2* rec = nullptr; T* Ftan = nullptr; T* Wtan = nullptr;
  T* raw = nullptr; T* rawdot = nullptr;
  T* Dl[3]; T* Vl[3]; T* Nl[3]; uint8_t* valid[3];
  double* Dhi[3] = {nullptr, nullptr, nullptr};   // FP32 runs: FP64 real part of the filtered depth
  T* Vm[3]; T* Nm[3]; T* Zm[3]; uint8_t* mvalid[3];
  double* partials = nullptr; int* lost = nullptr;
  MPose<D, Q>* Pcur; MPose<D, Q>* Pprev; MPose<D, Q>* Pprev2; MPose<D, Q>* Pinit; MPose<D, Q>* hist;
  KPose<T, D, Q>* Kcur; KPose<T, D, Q>* Kprev; KPose<T, D, Q>* Kq;
  int32_t* counters = nullptr;
  double* sums = nullptr; double* traj = nullptr; double* gt = nullptr;
  T* stage = nullptr;
  int* blist = nullptr; int* bcount = nullptr; uint8_t* bflags = nullptr;
  int* fcounts = nullptr; int* rhits = nullptr; int* rsamples = nullptr;
  T2* bracket = nullptr;
  float* cnn_in = nullptr; float* cnn_xi = nullptr; MPose<D, Q>* Pcand = nullptr;
  double* sums_net = nullptr; double* sums_cv = nullptr;
  xslam_cnn cnn = nullptr;
  T* tzmax = nullptr; T* czmax = nullptr; int* dframe = nullptr;
  // surfel map (map = XSLAM_MAP_SURFEL)
  bool surf = false;
  SurfMap<T> sm{};
  SurfCfg scfg{};
  unsigned long long* smap4 = nullptr; unsigned long long* smap1 = nullptr;
  uint8_t* sfresh = nullptr; int* sbcnt = nullptr; int* sboff = nullptr; int* supd = nullptr;
  int ntiles = 0;
  hipGraph_t graph = nullptr; hipGraphExec_t gexec = nullptr;
  bool use_graph = true;
  // launch shapes (none changes a result beyond the order of the FP64 ICP sums)
  int ray_bx = 16, ray_by = 16;
  int icp_grid[3] = {0, 0, 0};      // 0: one pixel per thread, at most kMaxIcpBlocks
  int fuse_grid = kFuseBlocks;

  // workgroups of any raycast tile of at least 64 threads:
  // ceil(W/bx) ceil(H/by) <= W H / 64 + W + H + 1
  static int ray_block_capacity(int w, int h) { return w * h / 64 + w + h + 1; }

  // ---- workspace plan ---------------------------------------------------
  static size_t plan(const xslam_config& c, int ndd, bool wtan, Engine* e, char* base) {
    Carver cv(base);
    const int64_t nv = int64_t(c.vol.dim[0]) * c.vol.dim[1] * c.vol.dim[2];
    const size_t n0 = size_t(c.cam.width) * c.cam.height;
    T2* rec = cv.take<T2>(nv);
    T* Ftan = NC > 1 ? cv.take<T>(size_t(NC - 1) * nv) : nullptr;
    T* Wtan = wtan ? cv.take<T>(nv) : nullptr;
    T* raw = cv.take<T>(n0);
    T* rawdot = ndd ? cv.take<T>(size_t(ndd) * n0) : nullptr;
    T *Dl[3], *Vl[3], *Nl[3], *Vm[3], *Nm[3], *Zm[3];
    uint8_t *vl[3], *mv[3];
    for (int l = 0; l < 3; ++l) {
      size_t n = size_t(c.cam.width >> l) * (c.cam.height >> l);
      Dl[l] = cv.take<T>(NC * n);
      Vl[l] = cv.take<T>(3 * NC * n);
      Nl[l] = cv.take<T>(3 * NC * n);
      vl[l] = cv.take<uint8_t>(n);
      Vm[l] = cv.take<T>(3 * NC * n);
      Nm[l] = cv.take<T>(3 * NC * n);
      Zm[l] = cv.take<T>(n);
      mv[l] = cv.take<uint8_t>(n);
    }
    double* dhi[3] = {nullptr, nullptr, nullptr};
    if (std::is_same<T, float>::value)
      for (int l = 0; l < 3; ++l) dhi[l] = cv.take<double>(size_t(c.cam.width >> l) * (c.cam.height >> l));
    // (real runs may use the Newton pass, whose partials are wider)
    double* partials = cv.take<double>(size_t(kMaxIcpBlocks) * ((D == 0 && Q == 0 && kNewtonNS > NS) ? kNewtonNS : NS));
    int* lost = cv.take<int>(1);
    MPose<D, Q>* P = cv.take<MPose<D, Q>>(4);
    MPose<D, Q>* hist = cv.take<MPose<D, Q>>(c.max_frames);
    KPose<T, D, Q>* K = cv.take<KPose<T, D, Q>>(3);
    int32_t* counters = cv.take<int32_t>(size_t(kCounters) * c.max_frames);
    double* sums = cv.take<double>(NS);
    double* traj = cv.take<double>(NC);
    double* gt = cv.take<double>(size_t(16) * c.max_frames);
    T* stage = cv.take<T>(kStageElems);
    const int nb = (c.vol.dim[0] / kBrick) * (c.vol.dim[1] / kBrick) * (c.vol.dim[2] / kBrick);
    int* blist = cv.take<int>(nb);
    int* bcount = cv.take<int>(1);
    uint8_t* bflags = cv.take<uint8_t>(nb);
    const int nt = ((c.cam.width + kTile - 1) / kTile) * ((c.cam.height + kTile - 1) / kTile);
    T* tzmax = cv.take<T>(nt);
    const int ncell = ((c.cam.width + kTile * kCell - 1) / (kTile * kCell)) *
                      ((c.cam.height + kTile * kCell - 1) / (kTile * kCell));
    T* czmax = cv.take<T>(ncell);
    const int nrb = ray_block_capacity(c.cam.width, c.cam.height);
    int* fcounts = cv.take<int>(kFuseBlocks);
    int* rhits = cv.take<int>(nrb);
    int* rsamples = cv.take<int>(nrb);
    T2* bracket = cv.take<T2>(n0);
    float* cnn_in = cv.take<float>(5 * (c.cam.width >> 3) * (c.cam.height >> 3));
    float* cnn_xi = cv.take<float>(8);
    MPose<D, Q>* Pcand = cv.take<MPose<D, Q>>(1);
    double* sums_net = cv.take<double>(NS);
    double* sums_cv = cv.take<double>(NS);
    int* dframe = cv.take<int>(1);
    // surfel map
    const bool sf = c.map == XSLAM_MAP_SURFEL;
    const size_t cap = sf ? size_t(c.surfel.capacity) : 0;
    const int nsb = sf ? int((n0 + kSurfScanBlock - 1) / kSurfScanBlock) : 0;
    const int nub = sf ? int(((c.cam.width + 15) / 16) * ((c.cam.height + 15) / 16)) : 0;
    T* sv = cv.take<T>(3 * NC * cap);
    T* sn = cv.take<T>(3 * NC * cap);
    T* sr = cv.take<T>(NC * cap);
    T* sc = cv.take<T>(NC * cap);
    int32_t* st = cv.take<int32_t>(cap);
    int* scount = cv.take<int>(sf ? 2 : 0);
    unsigned long long* m4 = cv.take<unsigned long long>(sf ? 16 * n0 : 0);
    unsigned long long* m1 = cv.take<unsigned long long>(sf ? n0 : 0);
    uint8_t* fr = cv.take<uint8_t>(sf ? n0 : 0);
    int* bcn = cv.take<int>(nsb);
    int* bof = cv.take<int>(nsb);
    int* bup = cv.take<int>(nub);
    if (e) {
      e->surf = sf;
      e->sm = SurfMap<T>{sv, sn, sr, sc, st, scount, sf ? scount + 1 : nullptr};
      e->smap4 = m4; e->smap1 = m1; e->sfresh = fr; e->sbcnt = bcn; e->sboff = bof; e->supd = bup;
    }
    if (e) {
      e->blist = blist; e->bcount = bcount; e->bflags = bflags; e->tzmax = tzmax; e->czmax = czmax;
      e->dframe = dframe;
      e->ntiles = nt;
      e->fcounts = fcounts; e->rhits = rhits; e->rsamples = rsamples; e->bracket = bracket;
      e->cnn_in = cnn_in; e->cnn_xi = cnn_xi; e->Pcand = Pcand; e->sums_net = sums_net; e->sums_cv = sums_cv;
      e->rec = rec; e->Ftan = Ftan; e->Wtan = Wtan; e->raw = raw; e->rawdot = rawdot;
      for (int l = 0; l < 3; ++l) {
        e->Dl[l] = Dl[l]; e->Vl[l] = Vl[l]; e->Nl[l] = Nl[l]; e->valid[l] = vl[l];
        e->Vm[l] = Vm[l]; e->Nm[l] = Nm[l]; e->Zm[l] = Zm[l]; e->mvalid[l] = mv[l];
      }
      e->partials = partials; e->lost = lost;
      for (int l = 0; l < 3; ++l) e->Dhi[l] = dhi[l];
      e->Pcur = P; e->Pprev = P + 1; e->Pprev2 = P + 2; e->Pinit = P + 3; e->hist = hist;
      e->Kcur = K; e->Kprev = K + 1; e->Kq = K + 2;
      e->counters = counters; e->sums = sums; e->traj = traj; e->gt = gt; e->stage = stage;
    }
    return cv.off;
  }

  // ---- error helpers ----------------------------------------------------
  int fail(int code, const std::string& msg) {
    C->err = msg;
    return code;
  }
  int check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(XSLAM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return XSLAM_OK;
  }
  int sync() {
    hipError_t e = hipStreamSynchronize(C->stream);
    if (e != hipSuccess) return fail(XSLAM_ERR_HIP, std::string("stream: ") + hipGetErrorString(e));
    return XSLAM_OK;
  }

  // kernel launch with optional event timing; cls: 0 measurement, 1 k_icp, 2 k_fuse, 3 k_raymarch,
  // 4 other, 5 k_icp_finish, 6 k_rayhit, 7 k_brick_cull
  // (timing: the dispatch itself stamps the event pair with its kernel's
  // start and end, so the pair brackets that kernel and nothing else)
  template <typename F> int launch(int cls, const char* what, F&& f) {
    Timer& tm = C->timer;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm.on && tm.next + 2 <= tm.pool.size()) {
      e0 = tm.pool[tm.next++];
      e1 = tm.pool[tm.next++];
    }
    tl_ev0 = e0;
    tl_ev1 = e1;
    f();
    tl_ev0 = tl_ev1 = nullptr;
    int rc = check(what);
    if (e1) tm.pending.push_back({cls, {e0, e1}});
    return rc;
  }

  // ---- construction -----------------------------------------------------
  int init(xslam_ctx_s* ctx, const double T0[16]) {
    C = ctx;
    const xslam_config& c = C->cfg;
    for (int l = 0; l < 3; ++l) {
      W[l] = c.cam.width >> l;
      H[l] = c.cam.height >> l;
      npx[l] = size_t(W[l]) * H[l];
    }
    nvox = int64_t(c.vol.dim[0]) * c.vol.dim[1] * c.vol.dim[2];
    // parameter jets
    auto pj = [&](double v, int param) {
      JD r = jconst<JD>(v);
      for (int d = 0; d < D; ++d)
        if (C->dirs[d].param == param) r.v[1 + d] = C->dirs[d].h;
      return r;
    };
    auto cast = [](const JD& x) { return jcast<T>(x); };
    kp.fx = cast(pj(c.cam.fx, XSLAM_P_FX));
    kp.fy = cast(pj(c.cam.fy, XSLAM_P_FY));
    kp.cx = cast(pj(c.cam.cx, XSLAM_P_CX));
    kp.cy = cast(pj(c.cam.cy, XSLAM_P_CY));
    kp.mu = cast(pj(c.vol.trunc, XSLAM_P_TRUNC));
    kp.wcap = cast(pj(c.vol.wcap, XSLAM_P_WCAP));
    kp.dgate2 = T(c.icp.dgate * c.icp.dgate);
    kp.cos_agate = T(std::cos(c.icp.agate_deg * M_PI / 180.0));
    kp.disc_delta = T(c.icp.disc_delta);
    kp.bil_is = T(1.0 / (2.0 * c.bilateral_sigma_px * c.bilateral_sigma_px));
    kp.bil_ir = T(1.0 / (2.0 * c.bilateral_sigma_m * c.bilateral_sigma_m));
    kp.pyr_gate = T(3.0 * c.bilateral_sigma_m);
    kp.bil_is_d = 1.0 / (2.0 * c.bilateral_sigma_px * c.bilateral_sigma_px);
    kp.bil_ir_d = 1.0 / (2.0 * c.bilateral_sigma_m * c.bilateral_sigma_m);
    kp.pyr_gate_d = 3.0 * c.bilateral_sigma_m;
    kp.voxel = T(c.vol.voxel);
    for (int a = 0; a < 3; ++a) {
      kp.half[a] = T(0.5 * c.vol.dim[a] * c.vol.voxel);
      kp.dim[a] = c.vol.dim[a];
      kp.nbr[a] = c.vol.dim[a] / kBrick;
    }
    nbrick = kp.nbr[0] * kp.nbr[1] * kp.nbr[2];
    kp.near_m = T(c.near_m);
    kp.bil_radius = c.bilateral_radius;
    kp.W = c.cam.width;
    kp.H = c.cam.height;
    kp.wcap_dir = -1;
    ndepth = 0;
    for (int d = 0; d < kMaxDirs; ++d) { kp.depth_plane[d] = -1; kp.depth_h[d] = T(0); }
    for (int d = 0; d < D; ++d) {
      if (C->dirs[d].param == XSLAM_P_WCAP) kp.wcap_dir = d;
      if (C->dirs[d].param == XSLAM_P_DEPTH) { kp.depth_plane[d] = ndepth++; kp.depth_h[d] = T(C->dirs[d].h); }
    }
    for (int l = 0; l < 3; ++l) omega[l] = pj(c.icp.level_w[l], XSLAM_P_ICPW0 + l);
    plan(c, ndepth, kp.wcap_dir >= 0, this, C->ws);
    // empty volume and maps
    int rc;
    if ((rc = fill<T>(reinterpret_cast<T*>(rec), T(0), 2 * nvox))) return rc;
    if (NC > 1 && (rc = fill<T>(Ftan, T(0), int64_t(NC - 1) * nvox))) return rc;
    if (Wtan && (rc = fill<T>(Wtan, T(0), nvox))) return rc;
    for (int l = 0; l < 3; ++l) {
      if ((rc = fill<uint8_t>(mvalid[l], 0, npx[l]))) return rc;
      if ((rc = fill<uint8_t>(valid[l], 0, npx[l]))) return rc;
    }
    if ((rc = fill<uint8_t>(bflags, 0, nbrick))) return rc;
    if ((rc = fill<int>(dframe, 0, 1))) return rc;
    if ((rc = fill<int>(bcount, 0, 1))) return rc;
    if ((rc = fill<int>(lost, 0, 1))) return rc;
    if ((rc = fill<int32_t>(counters, 0, int64_t(kCounters) * c.max_frames))) return rc;
    if (surf) {
      scfg.d_depth = c.surfel.d_depth;
      scfg.cos_norm = std::cos(c.surfel.d_norm_deg * M_PI / 180.0);
      scfg.d_dist = c.surfel.d_dist;
      scfg.two_s2 = 2.0 * c.surfel.sigma * c.surfel.sigma;
      scfg.c_stable = c.surfel.c_stable;
      scfg.cap = c.surfel.capacity;
      if ((rc = fill<int>(sm.count, 0, 2))) return rc;
    }
    // initial pose exp(xi_seed) T0, xi_seed = h on the pose directions
    JD xi[6];
    for (int a = 0; a < 6; ++a) xi[a] = pj(0.0, XSLAM_P_PHI_X + a);
    MPose<D, Q> T0p;
    for (int r = 0; r < 3; ++r) {
      for (int q = 0; q < 3; ++q) T0p.m[r * 3 + q] = jconst<JD>(T0[r * 4 + q]);
      T0p.m[9 + r] = jconst<JD>(T0[r * 4 + 3]);
    }
    MPose<D, Q> P0 = pose_mul(se3_exp<D, Q>(xi), T0p);
    if ((rc = put_pose(Pcur, Kcur, P0))) return rc;
    if ((rc = put_pose(Pprev, Kprev, P0))) return rc;
    if ((rc = put_pose(Pprev2, nullptr, P0))) return rc;
    if ((rc = put_pose(Pinit, nullptr, P0))) return rc;
    return sync();
  }

  template <typename P> int fill(P* p, P v, int64_t n) {
    if (n <= 0) return XSLAM_OK;
    int blocks = int(std::min<int64_t>((n + 255) / 256, 4096));
    return launch(4, "fill", [&] { XS_LAUNCH(k_fill<P>, dim3(blocks), dim3(256), 0, C->stream, p, v, n); });
  }

  int put_pose(MPose<D, Q>* dst, KPose<T, D, Q>* kdst, const MPose<D, Q>& P) {
    if (hipMemcpyAsync(dst, &P, sizeof(P), hipMemcpyHostToDevice, C->stream) != hipSuccess)
      return check("pose upload");
    if (kdst) {
      KPose<T, D, Q> K = to_kpose<T, double>(P);
      if (hipMemcpyAsync(kdst, &K, sizeof(K), hipMemcpyHostToDevice, C->stream) != hipSuccess)
        return check("pose upload");
    }
    return sync();  // the host structs above are stack temporaries
  }

  // ---- stages -------------------------------------------------------------
  int copy_inputs(const void* depth, const void* ddot) {
    if (!depth) return fail(XSLAM_ERR_ARG, "depth is NULL");
    if (ndepth > 0 && !ddot) return fail(XSLAM_ERR_ARG, "depth_dot required by a depth direction");
    hipError_t e = hipMemcpyAsync(raw, depth, npx[0] * sizeof(T), hipMemcpyDeviceToDevice, C->stream);
    if (e == hipSuccess && ndepth > 0)
      e = hipMemcpyAsync(rawdot, ddot, size_t(ndepth) * npx[0] * sizeof(T), hipMemcpyDeviceToDevice, C->stream);
    if (e != hipSuccess) return fail(XSLAM_ERR_HIP, std::string("input copy: ") + hipGetErrorString(e));
    return XSLAM_OK;
  }

  TrackBegin<T, D, Q> track_begin_args() const {
    return TrackBegin<T, D, Q>{Pcur, Pprev, Pprev2, Pinit, Kcur, Kprev, lost, counters, dframe, C->cfg.max_frames,
                               C->cfg.icp.init >= 1 ? 1 : 0};
  }

  // begin_track: the bilateral launch also starts the tracking of the frame
  // (k_track_begin's work, folded into the first launch of a tracked frame)
  // ---- stage descriptors: the arguments of each frame-step launch (the
  // solo launches below and the grouped ones take the same)
  GBilateral<T, D, Q> d_bilateral(bool begin_track) const {
    GBilateral<T, D, Q> a{kp, raw, rawdot, Dl[0], Dhi[0], TrackBegin<T, D, Q>{}};
    if (begin_track) a.tb = track_begin_args();
    return a;
  }
  dim3 g_level(int l) const { return dim3((W[l] + 15) / 16, (H[l] + 15) / 16); }
  GPyrdown<T, D, Q> d_pyrdown(int l) const {
    return GPyrdown<T, D, Q>{kp, Dl[l - 1], W[l - 1], H[l - 1], Dl[l], Dhi[l - 1], Dhi[l]};
  }
  GVertexNormal<T, D, Q> d_vertex_normal() const {
    VNLevels<T> lv;
    lv.first[0] = 0;
    for (int l = 0; l < 3; ++l) {
      lv.D[l] = Dl[l]; lv.Dhi[l] = Dhi[l]; lv.V[l] = Vl[l]; lv.N[l] = Nl[l]; lv.valid[l] = valid[l];
      lv.W[l] = W[l]; lv.H[l] = H[l];
      lv.tiles_x[l] = (W[l] + 15) / 16;
      lv.first[l + 1] = lv.first[l] + lv.tiles_x[l] * ((H[l] + 15) / 16);
    }
    return GVertexNormal<T, D, Q>{kp, lv};
  }

  int run_measure(bool begin_track = false) {
    int rc;
    const dim3 b(16, 16);
    const auto a = d_bilateral(begin_track);
    if ((rc = launch(0, "bilateral", [&] {
           XS_LAUNCH((k_bilateral<T, D, Q>), g_level(0), b, 0, C->stream, a.kp, a.depth, a.ddot, a.Dout, a.Dhi, a.tb);
         })))
      return rc;
    for (int l = 1; l < 3; ++l) {
      const auto p = d_pyrdown(l);
      if ((rc = launch(0, "pyrdown", [&] {
             XS_LAUNCH((k_pyrdown<T, D, Q>), g_level(l), b, 0, C->stream, p.kp, p.Din, p.Wi, p.Hi, p.Dout, p.Dhi_in,
                       p.Dhi_out);
           })))
        return rc;
    }
    const auto v = d_vertex_normal();
    if ((rc = launch(0, "vertex_normal", [&] {
           XS_LAUNCH((k_vertex_normal<T, D, Q>), dim3(v.lv.first[3]), b, 0, C->stream, v.kp, v.lv);
         })))
      return rc;
    measured = true;
    return XSLAM_OK;
  }

  int32_t* host_counter_row() { return counters + size_t(kCounters) * std::min(frame, C->cfg.max_frames - 1); }

  IcpArgs<T, D, Q> icp_args(int l, int iter_slot, int do_solve, double* sums_out = nullptr) const {
    IcpArgs<T, D, Q> a;
    a.V = Vl[l]; a.N = Nl[l]; a.valid = valid[l];
    a.Vm = Vm[l]; a.Nm = Nm[l]; a.Zm = Zm[l]; a.validm = mvalid[l];
    a.W = W[l]; a.H = H[l]; a.level = l; a.iter_slot = iter_slot; a.do_solve = do_solve;
    a.Kcur = Kcur; a.Kprev = Kprev; a.Pcur = Pcur; a.omega = omega[l]; a.update = C->cfg.icp.update;
    a.partials = partials; a.lost = lost; a.counters = counters; a.sums_out = sums_out ? sums_out : sums;
    a.frame = dframe; a.max_frames = C->cfg.max_frames;
    return a;
  }
  int icp_blocks(int l) const {
    return icp_grid[l] > 0 ? icp_grid[l]
                           : int(std::min<size_t>((npx[l] + kIcpThreads - 1) / kIcpThreads, kMaxIcpBlocks));
  }

  int run_icp_level(int l, int iter_slot, int do_solve, double* sums_out = nullptr) {
    const IcpArgs<T, D, Q> a = icp_args(l, iter_slot, do_solve, sums_out);
    const int blocks = icp_blocks(l);
    if (C->cfg.icp.solver >= 1) {
      if constexpr (D == 0 && Q == 0) {
        int rc = launch(1, "icp_newton", [&] {
          if (C->cfg.icp.solver == 1)
            XS_LAUNCH((k_icp_newton<T, D, Q, true>), dim3(blocks), dim3(kIcpThreads), 0, C->stream, kp, a);
          else
            XS_LAUNCH((k_icp_newton<T, D, Q, false>), dim3(blocks), dim3(kIcpThreads), 0, C->stream, kp, a);
        });
        if (rc) return rc;
        return launch(5, "icp_newton_finish", [&] {
          XS_LAUNCH((k_icp_newton_finish<T, D, Q>), dim3(1), dim3(256), 0, C->stream, a, blocks);
        });
      } else {
        return fail(XSLAM_ERR_UNSUPPORTED, "icp: the Newton solver needs a perturbation with no directions");
      }
    }
    int rc = launch(1, "icp", [&] {
      XS_LAUNCH((k_icp<T, D, Q>), dim3(blocks), dim3(kIcpThreads), 0, C->stream, kp, a);
    });
    if (rc) return rc;
    return launch(5, "icp_finish", [&] {
      XS_LAUNCH((k_icp_finish<T, D, Q>), dim3(1), dim3(kFinishThreads<T, D, Q>), 0, C->stream, a, blocks);
    });
  }

  // begun: the tracking of the frame was started by run_measure(true)
  int run_track(bool begun = false) {
    int rc;
    if (!measured) return fail(XSLAM_ERR_STATE, "track: no measured frame");
    if (!have_model) return fail(XSLAM_ERR_STATE, "track: no model maps (raycast first)");
    if (!begun && (rc = launch(4, "track_begin", [&] {
                    XS_LAUNCH((k_track_begin<T, D, Q>), dim3(1), dim3(64), 0, C->stream, track_begin_args());
                  })))
      return rc;
    if (C->cfg.icp.init == 2 && cnn && (rc = learned_init())) return rc;
    int slot = 0;
    for (int l = 2; l >= 0; --l)
      for (int it = 0; it < C->cfg.icp.iters[l]; ++it, ++slot)
        if ((rc = run_icp_level(l, slot, 1))) return rc;
    return XSLAM_OK;
  }

  // network input of the current measured frame and the model maps at pose K
  int enqueue_cnn_parts(const KPose<T, D, Q>* K, float* out_depth, float* out_model) {
    dim3 b(16, 16), g(((W[0] >> 3) + 15) / 16, ((H[0] >> 3) + 15) / 16);
    return launch(4, "cnn_parts", [&] {
      XS_LAUNCH((k_cnn_parts<T, D, Q>), g, b, 0, C->stream, kp, Dl[2], Nm[0], Zm[0], mvalid[0], K,
                         out_depth, out_model);
    });
  }

  // learned initial pose: network candidate vs previous / constant velocity,
  // judged by the mean squared residual of one level-2 association pass
  int learned_init() {
    int rc;
    const int n3 = (W[0] >> 3) * (H[0] >> 3);
    if ((rc = enqueue_cnn_parts(Kprev, cnn_in, cnn_in + n3))) return rc;
    if ((rc = xslam_cnn_forward(cnn, cnn_in, 1, cnn_xi))) return fail(rc, "learned init: network forward");
    if ((rc = launch(4, "init_candidates", [&] {
           XS_LAUNCH((k_init_candidates<T, D, Q>), dim3(1), dim3(64), 0, C->stream, Pprev, Pinit, cnn_xi,
                              Pcand, Pcur, Kcur);
         })))
      return rc;
    if ((rc = run_icp_level(2, 0, 0, sums_net))) return rc;
    if ((rc = launch(4, "set_current", [&] {
           XS_LAUNCH((k_set_current<T, D, Q>), dim3(1), dim3(64), 0, C->stream, Pinit, Pcur, Kcur);
         })))
      return rc;
    if ((rc = run_icp_level(2, 0, 0, sums_cv))) return rc;
    return launch(4, "choose_init", [&] {
      XS_LAUNCH((k_choose_init<T, D, Q>), dim3(1), dim3(64), 0, C->stream, sums_net, sums_cv, NS, Pcand,
                         Pinit, Pcur, Kcur, counters, dframe, C->cfg.max_frames);
    });
  }

  void drop_graph() {
    if (gexec) { hipGraphExecDestroy(gexec); gexec = nullptr; }
    if (graph) { hipGraphDestroy(graph); graph = nullptr; }
  }

  bool frame_graph() const override { return gexec != nullptr && !C->timer.on; }

  int set_launch(const xslam_launch& l) override {
    const int bx = l.ray_tile[0], by = l.ray_tile[1];
    if (bx < 1 || by < 1 || bx * by < 64 || bx * by > 256 || (bx * by) % 64 != 0)
      return fail(XSLAM_ERR_ARG, "launch: raycast tile x*y must be a multiple of 64 in [64, 256]");
    for (int i = 0; i < 3; ++i)
      if (l.icp_blocks[i] < 0 || l.icp_blocks[i] > kMaxIcpBlocks)
        return fail(XSLAM_ERR_ARG, "launch: ICP workgroups must be in [0, 1200]");
    if (l.fuse_blocks < 64 || l.fuse_blocks > kFuseBlocks)
      return fail(XSLAM_ERR_ARG, "launch: fusion workgroups must be in [64, 4096]");
    ray_bx = bx;
    ray_by = by;
    for (int i = 0; i < 3; ++i) icp_grid[i] = l.icp_blocks[i];
    fuse_grid = l.fuse_blocks;
    drop_graph();
    return XSLAM_OK;
  }

  int get_launch(xslam_launch* l) override {
    l->ray_tile[0] = ray_bx;
    l->ray_tile[1] = ray_by;
    for (int i = 0; i < 3; ++i)
      l->icp_blocks[i] = icp_grid[i] > 0 ? icp_grid[i]
                                         : int(std::min<size_t>((npx[i] + kIcpThreads - 1) / kIcpThreads, kMaxIcpBlocks));
    l->fuse_blocks = fuse_grid;
    l->reserved[0] = l->reserved[1] = 0;
    return XSLAM_OK;
  }

  // mean time (ms) of reps runs of f after one untimed run, HIP events on the stream
  // GPU time of reps back-to-back calls of f, captured into a graph and
  // replayed: eagerly launched short kernels (an ICP pass is two launches of
  // ~10 us) would time the host's launch rate as much as the kernels
  template <typename F> int time_graph_ms(int reps, double* ms, F&& f) {
    // (the legacy null stream cannot be captured: time eager launches there)
    if (C->stream == nullptr) return time_ms(reps, ms, f);
    int rc = f();   // warm-up, eager
    if (rc) return rc;
    if (hipStreamBeginCapture(C->stream, hipStreamCaptureModeRelaxed) != hipSuccess) return check("autotune capture");
    for (int r = 0; r < reps && !rc; ++r) rc = f();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(C->stream, &g);
    if (rc || e != hipSuccess || !g) {
      if (g) hipGraphDestroy(g);
      return rc ? rc : check("autotune capture");
    }
    hipGraphExec_t ge = nullptr;
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
      hipGraphDestroy(g);
      return check("autotune graph");
    }
    hipGraphDestroy(g);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = check("autotune events");
    if (!rc && hipGraphLaunch(ge, C->stream) != hipSuccess) rc = check("autotune graph launch");   // warm
    if (!rc) hipEventRecord(e0, C->stream);
    if (!rc && hipGraphLaunch(ge, C->stream) != hipSuccess) rc = check("autotune graph launch");
    if (!rc) hipEventRecord(e1, C->stream);
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = check("autotune sync");
    float t = 0.f;
    if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = check("autotune timing");
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipGraphExecDestroy(ge);
    *ms = double(t) / reps;
    return rc;
  }

  template <typename F> int time_ms(int reps, double* ms, F&& f) {
    int rc = f();
    if (rc) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return check("autotune events");
    if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); return check("autotune events"); }
    hipEventRecord(e0, C->stream);
    for (int r = 0; r < reps && !rc; ++r) rc = f();
    hipEventRecord(e1, C->stream);
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = check("autotune sync");
    float t = 0.f;
    if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = check("autotune timing");
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms = double(t) / reps;
    return rc;
  }

  int shape_key() const override { return int(sizeof(T)) * 10000 + D * 100 + Q; }
  GroupBase* new_group(EngineBase* const* es, int n, hipStream_t stream, int persist) override;

  int autotune(int reps, double* ms_out) override {
    if (!measured || !have_model) return fail(XSLAM_ERR_STATE, "autotune: needs a measured frame and model maps");
    if (reps < 1 || reps > 1000) return fail(XSLAM_ERR_ARG, "autotune: reps in [1, 1000]");
    if (gexec) drop_graph();
    int rc = sync();
    if (rc) return rc;
    const bool timing = C->timer.on;
    C->timer.on = false;
    // raycast tile
    static const int tiles[][2] = {{16, 16}, {32, 8}, {8, 32}, {64, 4}, {16, 8}, {32, 4}, {64, 2},
                                   {8, 8},   {16, 4}, {32, 2}, {64, 1}};
    double best_ray = surf ? 0.0 : 1e30;
    int bbx = ray_bx, bby = ray_by;
    for (auto& t : tiles) {
      if (surf) break;                 // the surfel map renders no raycast
      ray_bx = t[0];
      ray_by = t[1];
      double ms = 0;
      if ((rc = time_ms(reps, &ms, [&] { return run_raycast(); }))) break;
      if (ms < best_ray) { best_ray = ms; bbx = t[0]; bby = t[1]; }
    }
    ray_bx = bbx;
    ray_by = bby;
    if (!rc && !surf) rc = run_raycast();   // the model maps again with the chosen tile (same values)
    // ICP grid per level (sums only): the candidates are close, so each is
    // timed in 3 interleaved rounds and its best round counts, and a smaller
    // grid (more pixels per thread) replaces a larger one only when it is 5%
    // faster: in frame steps the one-pixel-per-thread grids of levels 1 and 2
    // ran 30-40% faster than the smaller grids that won close timings here
    double best_icp[3] = {1e30, 1e30, 1e30};
    static const int grids[] = {0, 960, 768, 512, 384, 256, 192, 128, 96, 64, 32};   // 0: one pixel per thread
    constexpr int ng = int(sizeof(grids) / sizeof(grids[0]));
    for (int l = 0; l < 3 && !rc; ++l) {
      const int full = int(std::min<size_t>((npx[l] + kIcpThreads - 1) / kIcpThreads, kMaxIcpBlocks));
      double cand_ms[ng];
      for (int c = 0; c < ng; ++c) cand_ms[c] = 1e30;
      for (int round = 0; round < 3 && !rc; ++round)
        for (int c = 0; c < ng && !rc; ++c) {
          const int gsz = grids[c] == 0 ? full : grids[c];
          if (gsz > full || (c > 0 && gsz == full)) continue;
          icp_grid[l] = gsz;
          double ms = 0;
          if ((rc = time_graph_ms(reps, &ms, [&] { return run_icp_level(l, 0, 0, sums); }))) break;
          cand_ms[c] = std::min(cand_ms[c], ms);
        }
      int bestg = icp_grid[l];
      for (int c = 0; c < ng; ++c)   // grids[] runs from the largest to the smallest
        if (cand_ms[c] < 0.95 * best_icp[l]) {
          best_icp[l] = cand_ms[c];
          bestg = grids[c] == 0 ? full : grids[c];
        }
      icp_grid[l] = bestg;
    }
    C->timer.on = timing;
    if (!rc) rc = sync();
    if (ms_out) {
      ms_out[0] = best_ray;
      for (int l = 0; l < 3; ++l) ms_out[1 + l] = best_icp[l];
    }
    return rc;
  }

  int set_cnn(xslam_cnn c) override {
    cnn = c;
    drop_graph();
    use_graph = true;
    return XSLAM_OK;
  }

  int cnn_parts(float* depth, float* model) override {
    if (!measured || !have_model) return fail(XSLAM_ERR_STATE, "cnn_parts: needs a measured frame and model maps");
    int rc = enqueue_cnn_parts(Kcur, depth, model);
    return rc ? rc : sync();
  }

  // lost fallback + pose history (tracked frames), reset of the brick list
  int post_track(bool tracked, bool store) {
    return launch(4, "post_track", [&] {
      XS_LAUNCH((k_post_track<T, D, Q>), dim3(1), dim3(64), 0, C->stream, Pcur, Pinit, Kcur,
                         tracked ? lost : nullptr, store ? hist : nullptr, dframe, C->cfg.max_frames, bcount);
    });
  }

  // fusion: per-tile depth bound, brick culling, list-driven update, brick
  // flags.  The brick count is reset by the end-of-tracking work, which the
  // first launch here does too (post_track(tracked, store) folded in).
  dim3 g_tile_zmax() const {
    const int ntx = (W[0] + kTile - 1) / kTile, nty = (H[0] + kTile - 1) / kTile;
    return dim3((ntx + kCell - 1) / kCell, (nty + kCell - 1) / kCell);
  }
  GTileZmax<T, D, Q> d_tile_zmax(bool tracked, bool store) const {
    const PostTrack<T, D, Q> post{Pcur, Pinit, Kcur, tracked ? lost : nullptr, store ? hist : nullptr,
                                  dframe, C->cfg.max_frames, bcount};
    return GTileZmax<T, D, Q>{Dl[0], W[0], H[0], tzmax, czmax, post};
  }
  GBrickCull<T, D, Q> d_brick_cull() const {
    return GBrickCull<T, D, Q>{kp, Kcur, tzmax, czmax, nbrick, blist, bcount, lost};
  }
  int fuse_blocks() const { return std::min(nbrick, fuse_grid); }
  GFuse<T, D, Q> d_fuse() const {
    return GFuse<T, D, Q>{kp, Kcur, Dl[0], rec, Ftan, Wtan, lost, nvox, blist, bcount, fcounts};
  }
  // (the brick flags' workgroup 0 also sums the fusion counts)
  GBrickFlags<T> d_brick_flags() const {
    return GBrickFlags<T>{rec, bflags, blist, bcount, nbrick, fcounts, fuse_blocks(), counters, dframe,
                          C->cfg.max_frames};
  }

  GBrickApron<T> d_brick_apron() const { return GBrickApron<T>{bflags, kp.nbr[0], kp.nbr[1], kp.nbr[2]}; }
  dim3 g_brick_apron() const { return dim3((nbrick + 255) / 256); }
  int run_brick_apron() {
    const auto a = d_brick_apron();
    return launch(4, "brick_apron", [&] {
      XS_LAUNCH(k_brick_apron<T>, g_brick_apron(), dim3(256), 0, C->stream, a.flags, a.nbx, a.nby, a.nbz);
    });
  }

  int run_fuse(bool tracked, bool store) {
    int rc;
    const auto z = d_tile_zmax(tracked, store);
    if ((rc = launch(4, "tile_zmax", [&] {
           XS_LAUNCH((k_tile_zmax<T, D, Q>), g_tile_zmax(), dim3(256), 0, C->stream, z.D0, z.W, z.H, z.tmax, z.cmax,
                     z.post);
         })))
      return rc;
    const auto c = d_brick_cull();
    if ((rc = launch(7, "brick_cull", [&] {
           XS_LAUNCH((k_brick_cull<T, D, Q>), dim3((nbrick + 255) / 256), dim3(256), 0, C->stream, c.kp, c.Kk,
                     c.tmax, c.cmax, c.nbrick, c.list, c.count, c.lost);
         })))
      return rc;
    const int g = fuse_blocks();
    const auto f = d_fuse();
    if ((rc = launch(2, "fuse", [&] {
           XS_LAUNCH((k_fuse<T, D, Q>), dim3(g), dim3(kBrickVox), 0, C->stream, f.kp, f.Kk, f.Df, f.rec, f.Ftan,
                     f.Wtan, f.lost, f.nvox, f.list, f.count, f.block_counts);
         })))
      return rc;
    const auto bf = d_brick_flags();
    if ((rc = launch(4, "brick_flags", [&] {
           XS_LAUNCH(k_brick_flags<T>, dim3(g), dim3(kBrickVox), 0, C->stream, bf.rec, bf.flags, bf.list, bf.count,
                     bf.nbrick, bf.fcounts, bf.nf, bf.counter_base, bf.frame, bf.max_frames);
         })))
      return rc;
    return run_brick_apron();
  }

  // surfel map: index map at 4x, association and update, insertion in pixel
  // order (predicated on the device lost flag)
  int run_surf_update() {
    int rc;
    const int cap = scfg.cap;
    const int64_t n0 = int64_t(npx[0]);
    if ((rc = fill<unsigned long long>(smap4, kSurfEmpty, 16 * n0))) return rc;
    if ((rc = launch(4, "surf_project4", [&] {
           XS_LAUNCH((k_surf_project<T, D, Q>), dim3((cap + 255) / 256), dim3(256), 0, C->stream, kp, Kcur, sm, cap,
                     4, -1e300, smap4);
         })))
      return rc;
    const dim3 b(16, 16), g((W[0] + 15) / 16, (H[0] + 15) / 16);
    if ((rc = launch(2, "surf_assoc", [&] {
           XS_LAUNCH((k_surf_assoc<T, D, Q>), g, b, 0, C->stream, kp, Kcur, Vl[0], Nl[0], valid[0], sm, scfg, smap4,
                     sfresh, lost, dframe, supd);
         })))
      return rc;
    const int nsb = int((n0 + kSurfScanBlock - 1) / kSurfScanBlock);
    if ((rc = launch(4, "surf_count", [&] {
           XS_LAUNCH(k_surf_count<T>, dim3(nsb), dim3(kSurfScanBlock), 0, C->stream, sfresh, int(n0), sbcnt);
         })))
      return rc;
    if ((rc = launch(4, "surf_scan", [&] {
           XS_LAUNCH(k_surf_scan<T>, dim3(1), dim3(1024), 0, C->stream, sbcnt, nsb, sboff, supd, int(g.x * g.y),
                     sm.count, sm.base, cap, counters, dframe, C->cfg.max_frames);
         })))
      return rc;
    return launch(4, "surf_insert", [&] {
      XS_LAUNCH((k_surf_insert<T, D, Q>), dim3(nsb), dim3(kSurfScanBlock), 0, C->stream, kp, Kcur, Vl[0], Nl[0],
                sfresh, sboff, sm, cap, dframe);
    });
  }

  // surfel map: the model maps (levels 0-2) from the nearest stable surfel
  // per pixel at the current pose; end_frame as in run_raycast
  int run_surf_predict(bool end_frame = false) {
    int rc;
    const int cap = scfg.cap;
    if ((rc = fill<unsigned long long>(smap1, kSurfEmpty, int64_t(npx[0])))) return rc;
    if ((rc = launch(3, "surf_project1", [&] {
           XS_LAUNCH((k_surf_project<T, D, Q>), dim3((cap + 255) / 256), dim3(256), 0, C->stream, kp, Kcur, sm, cap,
                     1, scfg.c_stable, smap1);
         })))
      return rc;
    MapsOut<T, D, Q> o;
    for (int l = 0; l < 3; ++l) { o.V[l] = Vm[l]; o.N[l] = Nm[l]; o.Z[l] = Zm[l]; o.valid[l] = mvalid[l]; }
    const dim3 b(16, 16), g((W[0] + 15) / 16, (H[0] + 15) / 16);
    if ((rc = launch(6, "surf_maps", [&] {
           XS_LAUNCH((k_surf_maps<T, D, Q>), g, b, 0, C->stream, kp, Kcur, sm, cap, smap1, o, rhits);
         })))
      return rc;
    const int nrb = int(g.x * g.y);
    rc = launch(4, "sum_counts", [&] {
      XS_LAUNCH(k_sum_counts<T>, dim3(1), dim3(1024), 0, C->stream, rhits, nrb, nullptr, 0, counters, dframe,
                C->cfg.max_frames, 2, 31, nullptr, 0, end_frame ? dframe : nullptr);
    });
    if (!rc) have_model = true;
    return rc;
  }

  int all_brick_flags() {
    const int g = std::min(nbrick, 4096);
    int rc = launch(4, "brick_flags_all", [&] {
      XS_LAUNCH(k_brick_flags<T>, dim3(g), dim3(kBrickVox), 0, C->stream, rec, bflags, nullptr, nullptr,
                         nbrick, nullptr, 0, nullptr, nullptr, 0);
    });
    if (!rc) rc = run_brick_apron();
    return rc ? rc : sync();
  }

  // end_frame: the counter sums also advance the frame index (the frame's
  // last launch)
  // raycast tile grid for a tile of bx x by threads
  dim3 g_ray(int bx, int by) const { return dim3((W[0] + bx - 1) / bx, (H[0] + by - 1) / by); }
  GRaymarch<T, D, Q> d_raymarch() const { return GRaymarch<T, D, Q>{kp, Kcur, rec, bflags, bracket, rsamples}; }
  GRayhit<T, D, Q> d_rayhit() const {
    MapsOut<T, D, Q> o;
    for (int l = 0; l < 3; ++l) { o.V[l] = Vm[l]; o.N[l] = Nm[l]; o.Z[l] = Zm[l]; o.valid[l] = mvalid[l]; }
    return GRayhit<T, D, Q>{kp, Kcur, rec, Ftan, nvox, bracket, o, rhits};
  }
  // the raycast's hit and sample counts; end_frame: also advance the frame index
  GSumCounts<T> d_ray_sum(int nrb, bool end_frame) const {
    return GSumCounts<T>{rhits, nrb, rsamples, nrb, counters, dframe, C->cfg.max_frames, 2, 31, nullptr, 0,
                         end_frame ? dframe : nullptr};
  }

  int run_raycast(bool end_frame = false) {
    const dim3 b(ray_bx, ray_by), g = g_ray(ray_bx, ray_by);
    const auto m = d_raymarch();
    int rc = launch(3, "raymarch", [&] {
      XS_LAUNCH((k_raymarch<T, D, Q>), g, b, 0, C->stream, m.kp, m.Kk, m.rec, m.flags, m.bracket, m.block_samples);
    });
    if (rc) return rc;
    const auto h = d_rayhit();
    rc = launch(6, "rayhit", [&] {
      XS_LAUNCH((k_rayhit<T, D, Q>), g, b, 0, C->stream, h.kp, h.Kk, h.rec, h.Ftan, h.nvox, h.bracket, h.out,
                h.block_hits);
    });
    if (rc) return rc;
    const auto s = d_ray_sum(int(g.x * g.y), end_frame);
    rc = launch(4, "sum_counts", [&] {
      XS_LAUNCH(k_sum_counts<T>, dim3(1), dim3(1024), 0, C->stream, s.a, s.n, s.b, s.nb, s.counter_base, s.frame,
                s.max_frames, s.slot_a, s.slot_b, s.extra, s.slot_extra, s.advance);
    });
    if (!rc) have_model = true;
    return rc;
  }


  int reset_frame_flags() {
    int rc = fill<int>(lost, 0, 1);
    if (!rc) rc = fill<int32_t>(host_counter_row(), 0, kCounters);
    return rc;
  }

  // the device work of one tracked frame (captured once into a graph)
  int enqueue_tracked_frame() {
    int rc;
    if ((rc = run_measure(true))) return rc;
    if ((rc = run_track(true))) return rc;
    if (surf) {
      if ((rc = post_track(true, true))) return rc;
      if ((rc = run_surf_update())) return rc;
      return run_surf_predict(true);
    }
    if ((rc = run_fuse(true, true))) return rc;
    return run_raycast(true);
  }

  // ---- EngineBase ---------------------------------------------------------
  int measure(const void* depth, const void* ddot) override {
    int rc = copy_inputs(depth, ddot);
    return rc ? rc : run_measure();
  }

  int integrate(const double* pose) override {
    int rc;
    if (!measured) return fail(XSLAM_ERR_STATE, "integrate: no measured frame");
    if (pose && (rc = set_real_pose(pose))) return rc;
    if ((rc = fill<int>(lost, 0, 1))) return rc;
    return surf ? run_surf_update() : run_fuse(false, false);
  }

  int raycast(const double* pose, void* vmap, void* nmap) override {
    int rc;
    if (pose && (rc = set_real_pose(pose))) return rc;
    if ((rc = surf ? run_surf_predict() : run_raycast())) return rc;
    size_t bytes = size_t(3) * NC * npx[0] * sizeof(T);
    if (vmap && hipMemcpyAsync(vmap, Vm[0], bytes, hipMemcpyDeviceToDevice, C->stream) != hipSuccess)
      return check("vmap copy");
    if (nmap && hipMemcpyAsync(nmap, Nm[0], bytes, hipMemcpyDeviceToDevice, C->stream) != hipSuccess)
      return check("nmap copy");
    return XSLAM_OK;
  }

  int track() override {
    int rc = run_track();
    if (rc) return rc;
    return post_track(true, true);
  }

  int step(const void* depth, const void* ddot) override {
    int rc;
    if (frame >= C->cfg.max_frames) return fail(XSLAM_ERR_STATE, "step: max_frames reached");
    if ((rc = copy_inputs(depth, ddot))) return rc;
    if (frame == 0) {
      if ((rc = reset_frame_flags())) return rc;
      if ((rc = run_measure())) return rc;
      if (surf) {
        if ((rc = post_track(false, true))) return rc;
        if ((rc = run_surf_update())) return rc;
        if ((rc = run_surf_predict(true))) return rc;
      } else {
        if ((rc = run_fuse(false, true))) return rc;
        if ((rc = run_raycast(true))) return rc;
      }
    } else {
      if (!have_model) return fail(XSLAM_ERR_STATE, "step: no model maps");
      measured = true;
      if (use_graph && !C->timer.on) {
        if (!gexec) {
          if ((rc = capture())) return rc;
        }
        if (gexec) {
          if (hipGraphLaunch(gexec, C->stream) != hipSuccess) return check("graph launch");
        } else if ((rc = enqueue_tracked_frame())) {
          return rc;
        }
      } else if ((rc = enqueue_tracked_frame())) {
        return rc;
      }
    }
    frame += 1;
    return XSLAM_OK;
  }

  // capture the tracked-frame work into a graph; on failure keep eager launches
  int capture() {
    if (hipStreamBeginCapture(C->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
      hipGetLastError();
      use_graph = false;
      return XSLAM_OK;
    }
    int rc = enqueue_tracked_frame();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(C->stream, &g);
    if (rc || e != hipSuccess || !g) {
      hipGetLastError();
      if (g) hipGraphDestroy(g);
      use_graph = false;
      return rc;
    }
    if (hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      hipGetLastError();
      hipGraphDestroy(g);
      gexec = nullptr;
      use_graph = false;
      return XSLAM_OK;
    }
    graph = g;
    return XSLAM_OK;
  }

  ~Engine() override {
    if (gexec) hipGraphExecDestroy(gexec);
    if (graph) hipGraphDestroy(graph);
  }

  int icp_pass(int level, double* out) override {
    if (level < 0 || level > 2) return fail(XSLAM_ERR_ARG, "icp_pass: level");
    int rc;
    if ((rc = fill<int>(lost, 0, 1))) return rc;
    if ((rc = run_icp_level(level, 0, 0))) return rc;
    if (hipMemcpyAsync(out, sums, NS * sizeof(double), hipMemcpyDeviceToHost, C->stream) != hipSuccess)
      return check("sums copy");
    return sync();
  }

  // E, gradient, Hessian and count of the Newton objective of one pass at the
  // current pose (no solve); real runs only
  int icp_energy(int level, int through, double* out) override {
    if (level < 0 || level > 2) return fail(XSLAM_ERR_ARG, "icp_energy: level");
    if constexpr (D == 0 && Q == 0) {
      if (!measured) return fail(XSLAM_ERR_STATE, "icp_energy: no measured frame");
      if (!have_model) return fail(XSLAM_ERR_STATE, "icp_energy: no model maps");
      const int solver = C->cfg.icp.solver;
      C->cfg.icp.solver = through ? 2 : 1;
      int rc = fill<int>(lost, 0, 1);
      if (!rc) rc = run_icp_level(level, 0, 0);
      C->cfg.icp.solver = solver;
      if (rc) return rc;
      if (hipMemcpyAsync(out, sums, kNewtonOut * sizeof(double), hipMemcpyDeviceToHost, C->stream) != hipSuccess)
        return check("sums copy");
      return sync();
    } else {
      (void)out;
      return fail(XSLAM_ERR_UNSUPPORTED, "icp_energy: real runs only (a perturbation with no directions)");
    }
  }

  // relocalisation objective at the host pose T16 against the volume, with
  // the last measured frame as the query; real runs only
  int reloc_energy(const double* T16, double* out) override {
    if constexpr (D == 0 && Q == 0) {
      if (surf) return fail(XSLAM_ERR_UNSUPPORTED, "reloc_energy: needs the TSDF map");
      if (!measured) return fail(XSLAM_ERR_STATE, "reloc_energy: no measured frame");
      int rc = XSLAM_OK;
      const KPose<T, D, Q> Kh = to_kpose<T, double>(pose_from_host(T16));
      if (hipMemcpyAsync(Kq, &Kh, sizeof(Kh), hipMemcpyHostToDevice, C->stream) != hipSuccess)
        return check("pose upload");
      const int ntx = (W[0] + kTile - 1) / kTile, nty = (H[0] + kTile - 1) / kTile;
      const int ncx = (ntx + kCell - 1) / kCell, ncy = (nty + kCell - 1) / kCell;
      const PostTrack<T, D, Q> none{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr};
      if ((rc = launch(4, "tile_zmax", [&] {
             XS_LAUNCH((k_tile_zmax<T, D, Q>), dim3(ncx, ncy), dim3(256), 0, C->stream, Dl[0], W[0], H[0], tzmax,
                       czmax, none);
           })))
        return rc;
      if ((rc = launch(4, "reloc", [&] {
             XS_LAUNCH((k_reloc<T>), dim3(kRelocBlocks), dim3(kBrickVox), 0, C->stream, kp, Kq, Dl[0], tzmax, czmax,
                       bflags, rec, nbrick, partials);
           })))
        return rc;
      if ((rc = launch(4, "reloc_finish", [&] {
             XS_LAUNCH(k_reloc_finish<T>, dim3(1), dim3(1024), 0, C->stream, partials, sums);
           })))
        return rc;
      if (hipMemcpyAsync(out, sums, kRelocNS * sizeof(double), hipMemcpyDeviceToHost, C->stream) != hipSuccess)
        return check("sums copy");
      return sync();   // (Kh is a stack temporary)
    } else {
      (void)T16; (void)out;
      return fail(XSLAM_ERR_UNSUPPORTED, "reloc_energy: real runs only (a perturbation with no directions)");
    }
  }

  int traj_err(const double* gtp, int n, double* out) override {
    if (n <= 0 || n > frame || n > C->cfg.max_frames) return fail(XSLAM_ERR_ARG, "traj_err: n");
    if (hipMemcpyAsync(gt, gtp, size_t(16) * n * sizeof(double), hipMemcpyHostToDevice, C->stream) != hipSuccess)
      return check("gt upload");
    int rc = launch(4, "traj_err", [&] {
      XS_LAUNCH((k_traj_err<D, Q>), dim3(1), dim3(64), 0, C->stream, hist, gt, n, traj);
    });
    if (rc) return rc;
    if (hipMemcpyAsync(out, traj, NC * sizeof(double), hipMemcpyDeviceToHost, C->stream) != hipSuccess)
      return check("traj copy");
    return sync();
  }

  int frame_lost(int* l, bool stepped) override {
    int32_t row[kCounters];
    int f = std::min(stepped ? frame - 1 : frame, C->cfg.max_frames - 1);
    if (f < 0) { *l = 0; return XSLAM_OK; }
    if (hipMemcpyAsync(row, counters + size_t(kCounters) * f, sizeof(row), hipMemcpyDeviceToHost, C->stream) != hipSuccess)
      return check("counters copy");
    int rc = sync();
    *l = row[0];
    return rc;
  }

  // ---- poses <-> host ----------------------------------------------------
  static void pose_to_host(const MPose<D, Q>& P, double* out) {  // [NC][16]
    for (int c = 0; c < NC; ++c) {
      double* o = out + c * 16;
      for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) o[r * 4 + q] = P.m[r * 3 + q].v[c];
        o[r * 4 + 3] = P.m[9 + r].v[c];
      }
      o[12] = o[13] = o[14] = 0.0;
      o[15] = (c == 0) ? 1.0 : 0.0;
    }
  }
  static MPose<D, Q> pose_from_host(const double* in) {
    MPose<D, Q> P;
    for (int c = 0; c < NC; ++c) {
      const double* o = in + c * 16;
      for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) P.m[r * 3 + q].v[c] = o[r * 4 + q];
        P.m[9 + r].v[c] = o[r * 4 + 3];
      }
    }
    return P;
  }
  int set_real_pose(const double* T16) {
    std::vector<double> buf(size_t(16) * NC, 0.0);
    memcpy(buf.data(), T16, 16 * sizeof(double));
    return put_pose(Pcur, Kcur, pose_from_host(buf.data()));
  }
  int current_pose(double* out) override {
    MPose<D, Q> P;
    if (hipMemcpyAsync(&P, Pcur, sizeof(P), hipMemcpyDeviceToHost, C->stream) != hipSuccess) return check("pose copy");
    int rc = sync();
    if (!rc) pose_to_host(P, out);
    return rc;
  }

  // ---- get / set ----------------------------------------------------------
  int vol_xfer(bool get, int kind, int comp, T* host) {
    for (int64_t s0 = 0; s0 < nvox; s0 += kStageElems) {
      int64_t cnt = std::min<int64_t>(kStageElems, nvox - s0);
      int blocks = int((cnt + 255) / 256);
      int rc;
      if (get) {
        if ((rc = launch(4, "vol_gather", [&] {
               XS_LAUNCH(k_vol_gather<T>, dim3(blocks), dim3(256), 0, C->stream, rec, Ftan, Wtan, kind, comp,
                                  nvox, kp.dim[0], kp.dim[1], kp.nbr[0], kp.nbr[1], s0, cnt, stage);
             })))
          return rc;
        if (hipMemcpyAsync(host + s0, stage, cnt * sizeof(T), hipMemcpyDeviceToHost, C->stream) != hipSuccess)
          return check("vol copy");
        if ((rc = sync())) return rc;
      } else {
        if (hipMemcpyAsync(stage, host + s0, cnt * sizeof(T), hipMemcpyHostToDevice, C->stream) != hipSuccess)
          return check("vol copy");
        if ((rc = launch(4, "vol_scatter", [&] {
               XS_LAUNCH(k_vol_scatter<T>, dim3(blocks), dim3(256), 0, C->stream, rec, Ftan, Wtan, kind, comp,
                                  nvox, kp.dim[0], kp.dim[1], kp.nbr[0], kp.nbr[1], s0, cnt, stage);
             })))
          return rc;
        if ((rc = sync())) return rc;
      }
    }
    return XSLAM_OK;
  }

  int copy(bool get, void* host, const void* dev, size_t bytes) {
    hipError_t e = get ? hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, C->stream)
                       : hipMemcpyAsync(const_cast<void*>(dev), host, bytes, hipMemcpyHostToDevice, C->stream);
    if (e != hipSuccess) return fail(XSLAM_ERR_HIP, std::string("copy: ") + hipGetErrorString(e));
    return sync();
  }

  int xfer(bool get, int field, void* buf, size_t bytes) {
    auto need = [&](size_t b) { return bytes == b; };
    size_t tot3 = 0, tot1 = 0;
    for (int l = 0; l < 3; ++l) { tot1 += npx[l]; tot3 += 3 * npx[l]; }
    switch (field) {
      case XSLAM_F_POSE:
      case XSLAM_F_PREV_POSE: {
        if (!need(size_t(NC) * 16 * sizeof(double))) return fail(XSLAM_ERR_ARG, "pose: size");
        MPose<D, Q>* P = field == XSLAM_F_POSE ? Pcur : Pprev;
        KPose<T, D, Q>* K = field == XSLAM_F_POSE ? Kcur : Kprev;
        if (get) {
          MPose<D, Q> h;
          int rc = copy(true, &h, P, sizeof(h));
          if (!rc) pose_to_host(h, static_cast<double*>(buf));
          return rc;
        }
        return put_pose(P, K, pose_from_host(static_cast<const double*>(buf)));
      }
      case XSLAM_F_POSES: {
        if (get) {
          int nf = std::min(frame, C->cfg.max_frames);
          if (!need(size_t(nf) * NC * 16 * sizeof(double))) return fail(XSLAM_ERR_ARG, "poses: size");
          std::vector<MPose<D, Q>> h(nf);
          int rc = nf ? copy(true, h.data(), hist, nf * sizeof(MPose<D, Q>)) : 0;
          for (int k = 0; k < nf && !rc; ++k) pose_to_host(h[k], static_cast<double*>(buf) + size_t(k) * NC * 16);
          return rc;
        }
        // resume: rows 0 .. n-1 of the history, n = bytes / (NC*16 doubles)
        size_t row = size_t(NC) * 16 * sizeof(double);
        if (bytes % row || bytes / row > size_t(C->cfg.max_frames)) return fail(XSLAM_ERR_ARG, "poses: size");
        size_t nf = bytes / row;
        std::vector<MPose<D, Q>> h(nf);
        for (size_t k = 0; k < nf; ++k) h[k] = pose_from_host(static_cast<const double*>(buf) + k * NC * 16);
        return nf ? copy(false, h.data(), hist, nf * sizeof(MPose<D, Q>)) : XSLAM_OK;
      }
      case XSLAM_F_TSDF:
      case XSLAM_F_WEIGHT: {
        if (!need(size_t(NC) * nvox * sizeof(T))) return fail(XSLAM_ERR_ARG, "tsdf: size");
        T* h = static_cast<T*>(buf);
        bool isF = field == XSLAM_F_TSDF;
        for (int c = 0; c < NC; ++c) {
          T* plane = h + size_t(c) * nvox;
          int rc;
          if (c == 0) rc = vol_xfer(get, isF ? 0 : 1, 0, plane);
          else if (isF) rc = vol_xfer(get, 2, c - 1, plane);
          else if (c - 1 == kp.wcap_dir) rc = vol_xfer(get, 3, 0, plane);
          else {
            if (get) memset(plane, 0, nvox * sizeof(T));
            rc = 0;
          }
          if (rc) return rc;
        }
        return get ? XSLAM_OK : all_brick_flags();
      }
      case XSLAM_F_VMAP: case XSLAM_F_NMAP: {
        size_t b = size_t(3) * NC * npx[0] * sizeof(T);
        if (!need(b)) return fail(XSLAM_ERR_ARG, "map: size");
        int rc = copy(get, buf, field == XSLAM_F_VMAP ? Vm[0] : Nm[0], b);
        if (!rc && !get) rc = rebuild_model_pyramid();
        return rc;
      }
      case XSLAM_F_ZMAP: {
        if (!need(npx[0] * sizeof(T))) return fail(XSLAM_ERR_ARG, "zmap: size");
        int rc = copy(get, buf, Zm[0], npx[0] * sizeof(T));
        if (!rc && !get) rc = rebuild_model_pyramid();
        return rc;
      }
      case XSLAM_F_MVALID: {
        if (!need(npx[0])) return fail(XSLAM_ERR_ARG, "mvalid: size");
        int rc = copy(get, buf, mvalid[0], npx[0]);
        if (!rc && !get) { rc = rebuild_model_pyramid(); have_model = true; }
        return rc;
      }
      case XSLAM_F_MEAS_DEPTH: case XSLAM_F_MEAS_V: case XSLAM_F_MEAS_N: case XSLAM_F_MEAS_VALID: {
        size_t per = field == XSLAM_F_MEAS_DEPTH ? NC * sizeof(T) : field == XSLAM_F_MEAS_VALID ? 1 : 3 * NC * sizeof(T);
        if (!need(tot1 * per)) return fail(XSLAM_ERR_ARG, "meas: size");
        char* h = static_cast<char*>(buf);
        for (int l = 0; l < 3; ++l) {
          void* dev = field == XSLAM_F_MEAS_DEPTH ? (void*)Dl[l] : field == XSLAM_F_MEAS_V ? (void*)Vl[l]
                    : field == XSLAM_F_MEAS_N ? (void*)Nl[l] : (void*)valid[l];
          int rc = copy(get, h, dev, npx[l] * per);
          if (rc) return rc;
          h += npx[l] * per;
        }
        if (!get) measured = true;
        return XSLAM_OK;
      }
      case XSLAM_F_COUNTERS: {
        size_t row = size_t(kCounters) * sizeof(int32_t);
        if (get) {
          int nf = std::min(frame, C->cfg.max_frames);
          if (!need(size_t(nf) * row)) return fail(XSLAM_ERR_ARG, "counters: size");
          return nf ? copy(true, buf, counters, bytes) : XSLAM_OK;
        }
        // resume: rows 0 .. n-1 (the lost flags of the last two frames decide
        // whether constant velocity extrapolates)
        if (bytes % row || bytes / row > size_t(C->cfg.max_frames)) return fail(XSLAM_ERR_ARG, "counters: size");
        return bytes ? copy(false, buf, counters, bytes) : XSLAM_OK;
      }
      case XSLAM_F_SURF_V: case XSLAM_F_SURF_N: case XSLAM_F_SURF_R: case XSLAM_F_SURF_C: case XSLAM_F_SURF_T: {
        if (!surf) return fail(XSLAM_ERR_ARG, "surfel fields need the surfel map");
        const size_t cap = size_t(scfg.cap);
        const bool vec = field == XSLAM_F_SURF_V || field == XSLAM_F_SURF_N;
        const size_t per = field == XSLAM_F_SURF_T ? sizeof(int32_t) : (vec ? 3 : 1) * NC * sizeof(T);
        void* dev = field == XSLAM_F_SURF_V ? (void*)sm.v : field == XSLAM_F_SURF_N ? (void*)sm.n
                  : field == XSLAM_F_SURF_R ? (void*)sm.r : field == XSLAM_F_SURF_C ? (void*)sm.c : (void*)sm.t;
        if (get) {
          if (!need(cap * per)) return fail(XSLAM_ERR_ARG, "surfels: size");
          return copy(true, buf, dev, cap * per);
        }
        // set: the leading m entries of each plane ([planes][m] on the host)
        const size_t planes = field == XSLAM_F_SURF_T ? 1 : (vec ? 3 : 1) * NC;
        const size_t esz = field == XSLAM_F_SURF_T ? sizeof(int32_t) : sizeof(T);
        if (bytes % (planes * esz) || bytes / (planes * esz) > cap) return fail(XSLAM_ERR_ARG, "surfels: size");
        const size_t m = bytes / (planes * esz);
        for (size_t q = 0; q < planes; ++q) {
          if (hipMemcpyAsync(static_cast<char*>(dev) + q * cap * esz, static_cast<const char*>(buf) + q * m * esz,
                             m * esz, hipMemcpyHostToDevice, C->stream) != hipSuccess)
            return check("surfels upload");
        }
        return sync();
      }
      case XSLAM_F_SURF_COUNT: {
        if (!surf) return fail(XSLAM_ERR_ARG, "surfel fields need the surfel map");
        if (!need(sizeof(int32_t))) return fail(XSLAM_ERR_ARG, "surfel count: size");
        if (get) return copy(true, buf, sm.count, sizeof(int32_t));
        const int m = *static_cast<const int32_t*>(buf);
        if (m < 0 || m > scfg.cap) return fail(XSLAM_ERR_ARG, "surfel count: range");
        int rc = fill<int>(sm.count, m, 1);
        return rc ? rc : sync();
      }
      case XSLAM_F_FRAME: {
        if (!need(sizeof(int32_t))) return fail(XSLAM_ERR_ARG, "frame: size");
        if (get) { *static_cast<int32_t*>(buf) = frame; return XSLAM_OK; }
        int f = *static_cast<const int32_t*>(buf);
        if (f < 0 || f > C->cfg.max_frames) return fail(XSLAM_ERR_ARG, "frame: range");
        frame = f;
        int rc = fill<int>(dframe, f, 1);
        return rc ? rc : sync();
      }
    }
    return fail(XSLAM_ERR_ARG, "unknown field");
  }

  // after a host write of level-0 model maps: levels 1, 2 by subsampling
  int rebuild_model_pyramid() {
    std::vector<T> V(3 * NC * npx[0]), N(3 * NC * npx[0]), Z(npx[0]);
    std::vector<uint8_t> M(npx[0]);
    int rc;
    if ((rc = copy(true, V.data(), Vm[0], V.size() * sizeof(T)))) return rc;
    if ((rc = copy(true, N.data(), Nm[0], N.size() * sizeof(T)))) return rc;
    if ((rc = copy(true, Z.data(), Zm[0], Z.size() * sizeof(T)))) return rc;
    if ((rc = copy(true, M.data(), mvalid[0], M.size()))) return rc;
    for (int l = 1; l < 3; ++l) {
      size_t nl = npx[l];
      std::vector<T> Vl_(3 * NC * nl), Nl_(3 * NC * nl), Zl(nl);
      std::vector<uint8_t> Ml(nl);
      for (int y = 0; y < H[l]; ++y)
        for (int x = 0; x < W[l]; ++x) {
          size_t s = size_t(y << l) * W[0] + (x << l), d = size_t(y) * W[l] + x;
          for (int c = 0; c < 3 * NC; ++c) {
            Vl_[c * nl + d] = V[c * npx[0] + s];
            Nl_[c * nl + d] = N[c * npx[0] + s];
          }
          Zl[d] = Z[s];
          Ml[d] = M[s];
        }
      if ((rc = copy(false, Vl_.data(), Vm[l], Vl_.size() * sizeof(T)))) return rc;
      if ((rc = copy(false, Nl_.data(), Nm[l], Nl_.size() * sizeof(T)))) return rc;
      if ((rc = copy(false, Zl.data(), Zm[l], Zl.size() * sizeof(T)))) return rc;
      if ((rc = copy(false, Ml.data(), mvalid[l], Ml.size()))) return rc;
    }
    return XSLAM_OK;
  }

  int get(int field, void* dst, size_t bytes) override { return xfer(true, field, dst, bytes); }
  int set(int field, const void* src, size_t bytes) override {
    return xfer(false, field, const_cast<void*>(src), bytes);
  }
};

// ---------------------------------------------------------------------------
// Grouped stepping of several contexts of one shape: the tracked-frame work of
// every member in one grid per stage (group.hpp), captured into a graph that
// is replayed until the set of stepping members changes.  A member's frame 0
// runs its own step.  The members' ICP passes are taken level by level
// (coarse first), pass by pass; a member with fewer iterations at a level
// sits out the passes it does not have.
template <typename T, int D, int Q>
struct GroupRun : GroupBase {
  using E = Engine<T, D, Q>;
  std::vector<E*> e;
  hipStream_t stream;
  int persist;
  int failed = -1;
  std::vector<char> ran_;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  // the built plan: its members, descriptor tables, launches and graph
  std::vector<int> built;
  std::vector<char> htab;
  char* dtab = nullptr;
  size_t dcap = 0;
  std::vector<std::function<void(const char*)>> launches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  GroupRun(EngineBase* const* es, int n, hipStream_t s, int p) : stream(s), persist(p) {
    for (int i = 0; i < n; ++i) e.push_back(static_cast<E*>(es[i]));
    ran_.assign(n, 0);
  }
  int init() {
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess) return XSLAM_ERR_HIP;
    return XSLAM_OK;
  }
  ~GroupRun() override {
    hipStreamSynchronize(stream);
    drop();
    if (dtab) hipFree(dtab);
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
  }
  void drop() {
    if (gexec) { hipGraphExecDestroy(gexec); gexec = nullptr; }
    if (graph) { hipGraphDestroy(graph); graph = nullptr; }
    built.clear();
  }
  int fail_at(int m, int code, const std::string& msg) {
    failed = m;
    e[m]->C->err = msg;
    return code;
  }

  // one grouped launch: the members' descriptors, their grids and the block
  template <class A>
  void stage(const std::vector<A>& d, const std::vector<dim3>& grids, dim3 block) {
    const size_t off = align_up(htab.size());
    htab.resize(off + d.size() * sizeof(A));
    memcpy(htab.data() + off, d.data(), d.size() * sizeof(A));
    GroupMap m{};
    m.n = int(d.size());
    int f = 0;
    for (int i = 0; i < m.n; ++i) {
      m.first[i] = f;
      m.gx[i] = int(grids[i].x);
      m.gy[i] = int(grids[i].y);
      const int cnt = m.gx[i] * m.gy[i];
      f += i + 1 < m.n ? (cnt + kGroupAlign - 1) / kGroupAlign * kGroupAlign : cnt;
    }
    m.first[m.n] = f;
    m.total = f;
    const int grid = persist > 0 ? std::min(f, persist) : f;
    hipStream_t s = stream;
    launches.push_back([m, grid, block, off, s](const char* base) {
      if (grid == m.total)
        hipLaunchKernelGGL(k_group_once<A>, dim3(grid), block, 0, s, reinterpret_cast<const A*>(base + off), m);
      else
        hipLaunchKernelGGL(k_group<A>, dim3(grid), block, 0, s, reinterpret_cast<const A*>(base + off), m);
    });
  }

  // the tracked-frame stages of the members mem (indices into e)
  void plan(const std::vector<int>& mem) {
    htab.clear();
    launches.clear();
    const size_t n = mem.size();
    auto each = [&](auto f) {
      using A = decltype(f(e[mem[0]]));
      std::vector<A> v;
      for (int m : mem) v.push_back(f(e[m]));
      return v;
    };
    auto grids = [&](auto f) {
      std::vector<dim3> v;
      for (int m : mem) v.push_back(f(e[m]));
      return v;
    };
    const dim3 b16(16, 16);
    stage(each([](E* x) { return x->d_bilateral(true); }), grids([](E* x) { return x->g_level(0); }), b16);
    for (int l = 1; l < 3; ++l)
      stage(each([l](E* x) { return x->d_pyrdown(l); }), grids([l](E* x) { return x->g_level(l); }), b16);
    stage(each([](E* x) { return x->d_vertex_normal(); }),
          grids([](E* x) { return dim3(x->d_vertex_normal().lv.first[3]); }), b16);
    std::vector<int> slot(n, 0);
    for (int l = 2; l >= 0; --l) {
      int most = 0;
      for (int m : mem) most = std::max(most, e[m]->C->cfg.icp.iters[l]);
      for (int it = 0; it < most; ++it) {
        std::vector<GIcp<T, D, Q>> pi;
        std::vector<GIcpFinish<T, D, Q>> pf;
        std::vector<dim3> gi, gf;
        for (size_t k = 0; k < n; ++k) {
          E* x = e[mem[k]];
          if (it >= x->C->cfg.icp.iters[l]) continue;
          const IcpArgs<T, D, Q> a = x->icp_args(l, slot[k]++, 1);
          pi.push_back(GIcp<T, D, Q>{x->kp, a});
          pf.push_back(GIcpFinish<T, D, Q>{a, x->icp_blocks(l)});
          gi.push_back(dim3(x->icp_blocks(l)));
          gf.push_back(dim3(1));
        }
        stage(pi, gi, dim3(kIcpThreads));
        stage(pf, gf, dim3(kFinishThreads<T, D, Q>));
      }
    }
    stage(each([](E* x) { return x->d_tile_zmax(true, true); }), grids([](E* x) { return x->g_tile_zmax(); }),
          dim3(256));
    stage(each([](E* x) { return x->d_brick_cull(); }), grids([](E* x) { return dim3((x->nbrick + 255) / 256); }),
          dim3(256));
    stage(each([](E* x) { return x->d_fuse(); }), grids([](E* x) { return dim3(x->fuse_blocks()); }), dim3(kBrickVox));
    stage(each([](E* x) { return x->d_brick_flags(); }), grids([](E* x) { return dim3(x->fuse_blocks()); }),
          dim3(kBrickVox));
    stage(each([](E* x) { return x->d_brick_apron(); }), grids([](E* x) { return x->g_brick_apron(); }), dim3(256));
    const int bx = e[mem[0]]->ray_bx, by = e[mem[0]]->ray_by;
    stage(each([](E* x) { return x->d_raymarch(); }), grids([&](E* x) { return x->g_ray(bx, by); }), dim3(bx, by));
    stage(each([](E* x) { return x->d_rayhit(); }), grids([&](E* x) { return x->g_ray(bx, by); }), dim3(bx, by));
    stage(each([&](E* x) {
            const dim3 g = x->g_ray(bx, by);
            return x->d_ray_sum(int(g.x * g.y), true);
          }),
          grids([](E*) { return dim3(1); }), dim3(1024));
  }

  int build(const std::vector<int>& mem) {
    drop();
    plan(mem);
    if (hipStreamSynchronize(stream) != hipSuccess) return fail_at(mem[0], XSLAM_ERR_HIP, "group: stream");
    if (htab.size() > dcap) {
      if (dtab) hipFree(dtab);
      dtab = nullptr;
      dcap = 0;
      if (hipMalloc(&dtab, htab.size()) != hipSuccess) {
        hipGetLastError();
        return fail_at(mem[0], XSLAM_ERR_HIP, "group: descriptor table allocation");
      }
      dcap = htab.size();
    }
    if (hipMemcpy(dtab, htab.data(), htab.size(), hipMemcpyHostToDevice) != hipSuccess)
      return fail_at(mem[0], XSLAM_ERR_HIP, "group: descriptor upload");
    built = mem;
    // capture; on failure the launches run eagerly
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed) == hipSuccess) {
      for (auto& f : launches) f(dtab);
      hipGraph_t g = nullptr;
      if (hipStreamEndCapture(stream, &g) == hipSuccess && g) {
        if (hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0) == hipSuccess) {
          graph = g;
        } else {
          gexec = nullptr;
          hipGraphDestroy(g);
        }
      }
    }
    hipGetLastError();
    return XSLAM_OK;
  }

  int failed_member() const override { return failed; }
  bool ran(int m) const override { return ran_[m] != 0; }
  float last_ms() override {
    if (!timed) return -1.f;
    float ms = -1.f;
    if (hipEventSynchronize(ev1) != hipSuccess || hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess) return -1.f;
    return ms;
  }

  int step(const void* const* depths, const void* const* ddots, const int32_t* active) override {
    failed = -1;
    timed = false;
    const int n = int(e.size());
    std::vector<int> solo, grp;
    for (int m = 0; m < n; ++m) {
      ran_[m] = 0;
      if (active && !active[m]) continue;
      E* x = e[m];
      if (!depths[m]) return fail_at(m, XSLAM_ERR_ARG, "depth is NULL");
      if (x->C->timer.on) return fail_at(m, XSLAM_ERR_STATE, "group: kernel timing is on");
      if (x->C->cfg.icp.init == 2 && x->cnn) return fail_at(m, XSLAM_ERR_UNSUPPORTED, "group: learned initialiser");
      if (x->frame >= x->C->cfg.max_frames) return fail_at(m, XSLAM_ERR_STATE, "step: max_frames reached");
      if (x->ndepth > 0 && !(ddots && ddots[m]))
        return fail_at(m, XSLAM_ERR_ARG, "depth_dot required by a depth direction");
      if (x->frame == 0) {
        solo.push_back(m);
      } else {
        if (!x->have_model) return fail_at(m, XSLAM_ERR_STATE, "step: no model maps");
        grp.push_back(m);
      }
    }
    if (solo.empty() && grp.empty()) return XSLAM_OK;
    hipEventRecord(ev0, stream);
    for (int m : solo) {
      const int rc = e[m]->step(depths[m], ddots ? ddots[m] : nullptr);
      if (rc) { failed = m; return rc; }
      ran_[m] = 1;
    }
    if (!grp.empty()) {
      // the frames' inputs, one copy launch (entries that are not 16-byte
      // aligned go through hipMemcpyAsync)
      CopyMap cm{};
      int64_t most = 0;
      auto add = [&](const void* src, void* dst, int64_t bytes) -> int {
        if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) | uintptr_t(bytes)) & 15) {
          return hipMemcpyAsync(dst, src, size_t(bytes), hipMemcpyDeviceToDevice, stream) == hipSuccess ? 0 : 1;
        }
        cm.src[cm.n] = src;
        cm.dst[cm.n] = dst;
        cm.bytes[cm.n] = bytes;
        cm.n += 1;
        most = std::max(most, bytes);
        return 0;
      };
      for (int m : grp) {
        E* x = e[m];
        if (add(depths[m], x->raw, int64_t(x->npx[0] * sizeof(T))) ||
            (x->ndepth > 0 && add(ddots[m], x->rawdot, int64_t(size_t(x->ndepth) * x->npx[0] * sizeof(T)))))
          return fail_at(m, XSLAM_ERR_HIP, "group: input copy");
      }
      if (cm.n) {
        const int gx = int(std::min<int64_t>(256, (most / 16 + 255) / 256));
        hipLaunchKernelGGL(k_group_copy<T>, dim3(gx, cm.n), dim3(256), 0, stream, cm);
      }
      if (grp != built) {
        const int rc = build(grp);
        if (rc) return rc;
      }
      if (gexec) {
        if (hipGraphLaunch(gexec, stream) != hipSuccess) {
          hipGetLastError();
          return fail_at(grp[0], XSLAM_ERR_HIP, "group: graph launch");
        }
      } else {
        for (auto& f : launches) f(dtab);
      }
      if (hipGetLastError() != hipSuccess) return fail_at(grp[0], XSLAM_ERR_HIP, "group: launch");
      for (int m : grp) {
        e[m]->measured = true;
        e[m]->frame += 1;
        ran_[m] = 1;
      }
    }
    hipEventRecord(ev1, stream);
    timed = true;
    return XSLAM_OK;
  }
};

template <typename T, int D, int Q>
GroupBase* Engine<T, D, Q>::new_group(EngineBase* const* es, int n, hipStream_t stream, int persist) {
  auto* g = new GroupRun<T, D, Q>(es, n, stream, persist);
  if (g->init()) {
    delete g;
    return nullptr;
  }
  return g;
}

template <typename T, int D, int Q>
EngineBase* make_engine(xslam_ctx_s* ctx, const double T0[16], int* rc) {
  auto* e = new Engine<T, D, Q>();
  *rc = e->init(ctx, T0);
  if (*rc) { delete e; return nullptr; }
  return e;
}
template <typename T, int D, int Q>
size_t engine_bytes(const xslam_config& c, int ndd, bool wtan) {
  return Engine<T, D, Q>::plan(c, ndd, wtan, nullptr, nullptr);
}

}  // namespace xs
