// C ABI of the frame step (declared in include/xslam.h): argument checks,
// dispatch to the engine of the context's (precision, D, Q) shape, timing.
#include <hip/hip_runtime.h>
#include <string.h>
#include <cmath>
#include <new>
#include <string>
#include <vector>
#include "ctx.hpp"
#include "combos.hpp"

namespace xsc {
void* cnn_stream(const xslam_cnn_s* h);   // cnn.hip
}

namespace xs {
constexpr int kMaxDirsApi = 16;
#define XS_DECL(T, D, Q, NAME)                                                      \
  EngineBase* make_##NAME(xslam_ctx_s* ctx, const double T0[16], int* rc);          \
  size_t bytes_##NAME(const xslam_config& c, int ndd, bool wtan);
XS_COMBOS(XS_DECL)
#undef XS_DECL

struct Combo {
  int prec, D, Q;
  EngineBase* (*make)(xslam_ctx_s*, const double*, int*);
  size_t (*bytes)(const xslam_config&, int, bool);
};
template <typename T> constexpr int prec_of();
template <> constexpr int prec_of<float>() { return XSLAM_C64; }
template <> constexpr int prec_of<double>() { return XSLAM_C128; }
#define XS_ROW(T, D, Q, NAME) {prec_of<T>(), D, Q, &make_##NAME, &bytes_##NAME},
static const Combo kCombos[] = {XS_COMBOS(XS_ROW)};
#undef XS_ROW

static const Combo* find_combo(int prec, int D, int Q) {
  for (const Combo& c : kCombos)
    if (c.prec == prec && c.D == D && c.Q == Q) return &c;
  return nullptr;
}

// Validate config and perturbation; on success fill D, Q, ndepth, wcap flag.
static int validate(const xslam_config* c, const xslam_perturbation* p, int* D, int* Q, int* ndd, bool* wtan,
                    std::string* err) {
  auto bad = [&](const char* m) { *err = m; return XSLAM_ERR_ARG; };
  if (!c) return bad("config is NULL");
  if (c->prec != XSLAM_C64 && c->prec != XSLAM_C128) return bad("prec");
  if (c->cam.width < 16 || c->cam.height < 16 || c->cam.width % 4 || c->cam.height % 4)
    return bad("image size must be >= 16 and a multiple of 4");
  if (!(c->cam.fx > 0 && c->cam.fy > 0)) return bad("focal lengths");
  for (int a = 0; a < 3; ++a)
    if (c->vol.dim[a] < 16 || c->vol.dim[a] % 8) return bad("volume dims must be >= 16 and multiples of 8");
  if ((int64_t)c->vol.dim[0] * c->vol.dim[1] * c->vol.dim[2] > (int64_t(1) << 31)) return bad("volume too large");
  if (!(c->vol.voxel > 0 && c->vol.trunc > 0 && c->vol.wcap >= 1)) return bad("volume parameters");
  for (int l = 0; l < 3; ++l)
    if (c->icp.iters[l] < 0 || c->icp.iters[l] > 64) return bad("icp iterations");
  if (c->icp.iters[0] + c->icp.iters[1] + c->icp.iters[2] > 25) return bad("icp iterations: at most 25 passes");
  if (!(c->icp.dgate > 0)) return bad("dgate");
  if (c->icp.init < 0 || c->icp.init > 2) return bad("icp.init must be 0, 1 or 2");
  if (c->icp.update < 0 || c->icp.update > 1) return bad("icp.update must be 0 or 1");
  if (c->icp.solver < 0 || c->icp.solver > 2) return bad("icp.solver must be 0, 1 or 2");
  if (c->icp.init == 2 && (c->cam.width % 64 || c->cam.height % 32 || c->cam.width / 8 != 80 || c->cam.height / 8 != 60))
    return bad("icp.init 2 (network) needs 640 x 480 depth (a 80 x 60 level-3 input)");
  if (c->bilateral_radius < 0 || c->bilateral_radius > 4) return bad("bilateral radius must be 0..4");
  if (c->bilateral_radius > 0 && !(c->bilateral_sigma_px > 0 && c->bilateral_sigma_m > 0)) return bad("bilateral sigmas");
  if (!(c->bilateral_sigma_m > 0)) return bad("bilateral_sigma_m gates the pyramid and must be > 0");
  if (c->max_frames < 1) return bad("max_frames");
  if (c->map != XSLAM_MAP_TSDF && c->map != XSLAM_MAP_SURFEL) return bad("map must be 0 (TSDF) or 1 (surfels)");
  if (c->map == XSLAM_MAP_SURFEL) {
    const xslam_surfel& sf = c->surfel;
    if (sf.capacity < 1 || sf.capacity > (1 << 28)) return bad("surfel capacity must be 1..2^28");
    if (!(sf.d_depth > 0 && sf.d_dist > 0 && sf.sigma > 0) || !(sf.d_norm_deg >= 0 && sf.d_norm_deg <= 180) ||
        !std::isfinite(sf.c_stable))
      return bad("surfel gates and sigma");
  }
  int nd = p ? p->n_dirs : 0, np = p ? p->n_pairs : 0;
  if (nd < 0 || nd > kMaxDirsApi) return bad("n_dirs must be 0..16");
  if (nd > 0 && !p->dirs) return bad("dirs is NULL");
  if (c->icp.solver >= 1 && (nd > 0 || np > 0))
    return bad("icp.solver 1 or 2 (Newton) needs a perturbation with no directions: the increment's six directions "
               "and their pairs fill the jet");
  if (np > 0 && !p->pairs) return bad("pairs is NULL");
  *ndd = 0;
  *wtan = false;
  int nw = 0;
  for (int d = 0; d < nd; ++d) {
    const xslam_dir& x = p->dirs[d];
    if (x.param < 0 || x.param >= XSLAM_P_COUNT) return bad("direction parameter");
    if (!(x.h > 0) || !std::isfinite(x.h)) return bad("direction step h must be > 0");
    if (c->prec == XSLAM_C64 && (x.h < 1e-30 || x.h > 1.0)) return bad("FP32 step h must be in [1e-30, 1]");
    if (x.param == XSLAM_P_DEPTH) ++*ndd;
    if (x.param == XSLAM_P_WCAP) { ++nw; *wtan = true; }
  }
  if (nw > 1) return bad("at most one weight-cap direction");
  // pairs: the full upper triangle over the first q directions, row-major
  int q = 0;
  while (q * (q + 1) / 2 < np) ++q;
  if (q * (q + 1) / 2 != np || q > nd) return bad("pairs must be the upper triangle over the first Q directions");
  int k = 0;
  for (int a = 0; a < q; ++a)
    for (int b = a; b < q; ++b, ++k)
      if (p->pairs[k].a != a || p->pairs[k].b != b) return bad("pairs must be listed as (a,b), a<=b<Q, row-major");
  if (c->prec == XSLAM_C64)
    for (int a = 0; a < q; ++a)
      if (p->dirs[a].h < 1e-15) return bad("FP32 second-order steps need h >= 1e-15 (h^2 must stay normal)");
  *D = nd;
  *Q = q;
  return XSLAM_OK;
}
}  // namespace xs

using namespace xs;

extern "C" {

int32_t xslam_components(const xslam_perturbation* p) {
  if (!p) return 1;
  return 1 + p->n_dirs + p->n_pairs;
}

size_t xslam_workspace_bytes(const xslam_config* cfg, const xslam_perturbation* pert) {
  int D, Q, ndd;
  bool wtan;
  std::string err;
  if (validate(cfg, pert, &D, &Q, &ndd, &wtan, &err)) return 0;
  const Combo* cb = find_combo(cfg->prec, D, Q);
  if (!cb) return 0;
  return cb->bytes(*cfg, ndd, wtan);
}

int xslam_create(const xslam_config* cfg, const xslam_perturbation* pert, void* dev_workspace, size_t bytes,
                 void* stream, const double T0[16], xslam_ctx* out) {
  if (!out) return XSLAM_ERR_ARG;
  *out = nullptr;
  int D, Q, ndd;
  bool wtan;
  std::string err;
  int rc = validate(cfg, pert, &D, &Q, &ndd, &wtan, &err);
  if (rc) return rc;
  if (!T0) return XSLAM_ERR_ARG;
  const Combo* cb = find_combo(cfg->prec, D, Q);
  if (!cb) return XSLAM_ERR_UNSUPPORTED;
  size_t need = cb->bytes(*cfg, ndd, wtan);
  if (!dev_workspace || bytes < need || (reinterpret_cast<uintptr_t>(dev_workspace) & 255)) return XSLAM_ERR_WORKSPACE;
  xslam_ctx_s* c = new (std::nothrow) xslam_ctx_s();
  if (!c) return XSLAM_ERR_ARG;
  c->cfg = *cfg;
  if (pert) {
    c->dirs.assign(pert->dirs, pert->dirs + pert->n_dirs);
    c->pairs.assign(pert->pairs, pert->pairs + pert->n_pairs);
  }
  c->D = D;
  c->Q = Q;
  c->NC = 1 + D + Q * (Q + 1) / 2;
  c->stream = static_cast<hipStream_t>(stream);
  c->ws = static_cast<char*>(dev_workspace);
  c->ws_bytes = bytes;
  hipGetDevice(&c->device);
  c->eng = cb->make(c, T0, &rc);
  if (!c->eng) {
    delete c;
    return rc ? rc : XSLAM_ERR_HIP;
  }
  *out = c;
  return XSLAM_OK;
}

#define XS_CTX_CHECK(ctx) \
  if (!(ctx) || !(ctx)->eng) return XSLAM_ERR_ARG

int xslam_measure(xslam_ctx ctx, const void* depth, const void* depth_dot) {
  XS_CTX_CHECK(ctx);
  return ctx->eng->measure(depth, depth_dot);
}

int xslam_integrate(xslam_ctx ctx, const void* depth, const void* depth_dot, const double* pose) {
  XS_CTX_CHECK(ctx);
  if (depth) {
    int rc = ctx->eng->measure(depth, depth_dot);
    if (rc) return rc;
  }
  return ctx->eng->integrate(pose);
}

int xslam_raycast(xslam_ctx ctx, const double* pose, void* vmap, void* nmap) {
  XS_CTX_CHECK(ctx);
  return ctx->eng->raycast(pose, vmap, nmap);
}

static int finish_pose(xslam_ctx ctx, double* pose_out, bool stepped) {
  if (!pose_out) return XSLAM_OK;
  int rc = ctx->eng->current_pose(pose_out);
  if (rc) return rc;
  int lost = 0;
  rc = ctx->eng->frame_lost(&lost, stepped);
  if (rc) return rc;
  return lost ? XSLAM_WARN_TRACK_LOST : XSLAM_OK;
}

int xslam_track(xslam_ctx ctx, const void* depth, const void* depth_dot, double* pose_out) {
  XS_CTX_CHECK(ctx);
  int rc = depth ? ctx->eng->measure(depth, depth_dot) : XSLAM_OK;
  if (rc) return rc;
  rc = ctx->eng->track();
  if (rc) return rc;
  return finish_pose(ctx, pose_out, false);
}

int xslam_step(xslam_ctx ctx, const void* depth, const void* depth_dot, double* pose_out) {
  XS_CTX_CHECK(ctx);
  int rc = ctx->eng->step(depth, depth_dot);
  if (rc) return rc;
  return finish_pose(ctx, pose_out, true);
}

int xslam_icp_pass(xslam_ctx ctx, int32_t level, double* sums_out) {
  XS_CTX_CHECK(ctx);
  if (!sums_out) return XSLAM_ERR_ARG;
  return ctx->eng->icp_pass(level, sums_out);
}

int xslam_icp_energy(xslam_ctx ctx, int32_t level, int32_t through, double* out) {
  XS_CTX_CHECK(ctx);
  if (!out || through < 0 || through > 1) return XSLAM_ERR_ARG;
  return ctx->eng->icp_energy(level, through, out);
}

int xslam_reloc_energy(xslam_ctx ctx, const double pose[16], double* out) {
  XS_CTX_CHECK(ctx);
  if (!pose || !out) return XSLAM_ERR_ARG;
  for (int k = 0; k < 16; ++k)
    if (!std::isfinite(pose[k])) return XSLAM_ERR_ARG;
  return ctx->eng->reloc_energy(pose, out);
}

int xslam_traj_err(xslam_ctx ctx, const double* gt_poses, int32_t n, double* out) {
  XS_CTX_CHECK(ctx);
  if (!gt_poses || !out) return XSLAM_ERR_ARG;
  return ctx->eng->traj_err(gt_poses, n, out);
}

int xslam_get(xslam_ctx ctx, int32_t field, void* dst, size_t bytes) {
  XS_CTX_CHECK(ctx);
  if (!dst) return XSLAM_ERR_ARG;
  return ctx->eng->get(field, dst, bytes);
}

int xslam_set(xslam_ctx ctx, int32_t field, const void* src, size_t bytes) {
  XS_CTX_CHECK(ctx);
  if (!src) return XSLAM_ERR_ARG;
  return ctx->eng->set(field, src, bytes);
}

int xslam_set_timing(xslam_ctx ctx, int32_t on) {
  XS_CTX_CHECK(ctx);
  Timer& t = ctx->timer;
  if (on && t.pool.empty()) {
    t.pool.resize(8192);
    for (auto& e : t.pool)
      if (hipEventCreate(&e) != hipSuccess) return XSLAM_ERR_HIP;
  }
  t.on = on != 0;
  return XSLAM_OK;
}

int xslam_kernel_times(xslam_ctx ctx, double ms_out[8], int64_t launches_out[8]) {
  XS_CTX_CHECK(ctx);
  Timer& t = ctx->timer;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return XSLAM_ERR_HIP;
  for (auto& p : t.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.second.first, p.second.second) != hipSuccess) return XSLAM_ERR_HIP;
    t.ms[p.first] += ms;
    t.launches[p.first] += 1;
  }
  t.pending.clear();
  t.next = 0;
  for (int i = 0; i < Timer::kClasses; ++i) {
    if (ms_out) ms_out[i] = t.ms[i];
    if (launches_out) launches_out[i] = t.launches[i];
  }
  return XSLAM_OK;
}

int xslam_ctx_set_cnn(xslam_ctx ctx, xslam_cnn cnn) {
  XS_CTX_CHECK(ctx);
  if (cnn && xsc::cnn_stream(cnn) != static_cast<void*>(ctx->stream)) {
    ctx->err = "set_cnn: the network was created on another stream than the context";
    return XSLAM_ERR_ARG;
  }
  return ctx->eng->set_cnn(cnn);
}

int xslam_cnn_parts(xslam_ctx ctx, float* depth_dev, float* model_dev) {
  XS_CTX_CHECK(ctx);
  if (!depth_dev || !model_dev) return XSLAM_ERR_ARG;
  return ctx->eng->cnn_parts(depth_dev, model_dev);
}

int xslam_set_launch(xslam_ctx ctx, const xslam_launch* shapes) {
  XS_CTX_CHECK(ctx);
  if (!shapes) return XSLAM_ERR_ARG;
  return ctx->eng->set_launch(*shapes);
}

int xslam_frame_graph(xslam_ctx ctx, int32_t* active) {
  XS_CTX_CHECK(ctx);
  if (!active) return XSLAM_ERR_ARG;
  *active = ctx->eng->frame_graph() ? 1 : 0;
  return XSLAM_OK;
}

int xslam_get_launch(xslam_ctx ctx, xslam_launch* out) {
  XS_CTX_CHECK(ctx);
  if (!out) return XSLAM_ERR_ARG;
  return ctx->eng->get_launch(out);
}

int xslam_autotune(xslam_ctx ctx, int32_t reps, xslam_launch* best, double* ms_out) {
  XS_CTX_CHECK(ctx);
  int rc = ctx->eng->autotune(reps, ms_out);
  if (!rc && best) rc = ctx->eng->get_launch(best);
  return rc;
}

int xslam_sync(xslam_ctx ctx) {
  XS_CTX_CHECK(ctx);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    ctx->err = std::string("stream: ") + hipGetErrorString(e);
    return XSLAM_ERR_HIP;
  }
  return XSLAM_OK;
}

struct xslam_batch_s {
  std::vector<xslam_ctx> ctx;
  std::vector<hipEvent_t> e0, e1;
  std::vector<char> ran;
  int32_t last_index = -1;
  // grouped batches: the groups and, per group, its members' context indices
  std::vector<xs::GroupBase*> groups;
  std::vector<std::vector<int>> members;
};

int xslam_batch_create(const xslam_ctx* ctxs, int32_t n, xslam_batch* out) {
  if (!ctxs || n < 1 || !out) return XSLAM_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !ctxs[i]->eng) return XSLAM_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return XSLAM_ERR_ARG;
  }
  auto* b = new xslam_batch_s;
  b->ctx.assign(ctxs, ctxs + n);
  b->e0.assign(n, nullptr);
  b->e1.assign(n, nullptr);
  b->ran.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    if (hipSetDevice(ctxs[i]->device) != hipSuccess || hipEventCreate(&b->e0[i]) != hipSuccess ||
        hipEventCreate(&b->e1[i]) != hipSuccess) {
      for (auto e : b->e0) if (e) hipEventDestroy(e);
      for (auto e : b->e1) if (e) hipEventDestroy(e);
      delete b;
      return XSLAM_ERR_HIP;
    }
  }
  *out = b;
  return XSLAM_OK;
}

int xslam_batch_create_grouped(const xslam_ctx* ctxs, int32_t n, int32_t persist, xslam_batch* out) {
  if (!ctxs || n < 1 || !out || persist < 0 || persist % xs::kGroupAlign) return XSLAM_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !ctxs[i]->eng) return XSLAM_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return XSLAM_ERR_ARG;
  }
  for (int i = 0; i < n; ++i) {
    const xslam_config& c = ctxs[i]->cfg;
    if (c.map != XSLAM_MAP_TSDF || c.icp.solver != 0) {
      ctxs[i]->err = "grouped batch: needs the TSDF map and the Gauss-Newton solver";
      return XSLAM_ERR_UNSUPPORTED;
    }
    if (ctxs[i]->device != ctxs[0]->device) {
      ctxs[i]->err = "grouped batch: contexts on different devices";
      return XSLAM_ERR_ARG;
    }
  }
  auto* b = new xslam_batch_s;
  b->ctx.assign(ctxs, ctxs + n);
  b->ran.assign(n, 0);
  // members by shape and stream, in context order, at most kGroupMax per group
  std::vector<char> taken(n, 0);
  int rc = XSLAM_OK;
  for (int i = 0; i < n && !rc; ++i) {
    if (taken[i]) continue;
    std::vector<int> mem;
    for (int j = i; j < n && int(mem.size()) < xs::kGroupMax; ++j)
      if (!taken[j] && ctxs[j]->eng->shape_key() == ctxs[i]->eng->shape_key() && ctxs[j]->stream == ctxs[i]->stream) {
        mem.push_back(j);
        taken[j] = 1;
      }
    std::vector<xs::EngineBase*> es;
    for (int j : mem) es.push_back(ctxs[j]->eng);
    hipSetDevice(ctxs[i]->device);
    xs::GroupBase* g = ctxs[i]->eng->new_group(es.data(), int(es.size()), ctxs[i]->stream, persist);
    if (!g) { rc = XSLAM_ERR_HIP; break; }
    b->groups.push_back(g);
    b->members.push_back(mem);
  }
  if (rc) {
    for (auto g : b->groups) delete g;
    delete b;
    return rc;
  }
  *out = b;
  return XSLAM_OK;
}

static int batch_step_grouped(xslam_batch b, const void* const* depths, const void* const* depth_dots,
                              const int32_t* active) {
  for (size_t k = 0; k < b->groups.size(); ++k) {
    const std::vector<int>& mem = b->members[k];
    std::vector<const void*> d(mem.size()), dd(mem.size());
    std::vector<int32_t> act(mem.size());
    for (size_t q = 0; q < mem.size(); ++q) {
      d[q] = depths[mem[q]];
      dd[q] = depth_dots ? depth_dots[mem[q]] : nullptr;
      act[q] = active ? active[mem[q]] : 1;
    }
    const int rc = b->groups[k]->step(d.data(), dd.data(), act.data());
    for (size_t q = 0; q < mem.size(); ++q) b->ran[mem[q]] = b->groups[k]->ran(int(q)) ? 1 : 0;
    if (rc) {
      const int f = b->groups[k]->failed_member();
      b->last_index = f >= 0 ? mem[f] : mem[0];
      return rc;
    }
  }
  return XSLAM_OK;
}

int xslam_batch_step(xslam_batch b, const void* const* depths, const void* const* depth_dots,
                     const int32_t* active) {
  if (!b || !depths) return XSLAM_ERR_ARG;
  b->last_index = -1;
  if (!b->groups.empty()) return batch_step_grouped(b, depths, depth_dots, active);
  const int n = int(b->ctx.size());
  for (int i = 0; i < n; ++i) {
    b->ran[i] = 0;
    if (active && !active[i]) continue;
    xslam_ctx c = b->ctx[i];
    hipEventRecord(b->e0[i], c->stream);
    int rc = c->eng->step(depths[i], depth_dots ? depth_dots[i] : nullptr);
    hipEventRecord(b->e1[i], c->stream);
    if (rc) {
      b->last_index = i;
      return rc;
    }
    b->ran[i] = 1;
  }
  return XSLAM_OK;
}

int xslam_batch_latency(xslam_batch b, float* ms_out) {
  if (!b || !ms_out) return XSLAM_ERR_ARG;
  if (!b->groups.empty()) {
    for (size_t k = 0; k < b->groups.size(); ++k) {
      const float ms = b->groups[k]->last_ms();
      for (int i : b->members[k]) ms_out[i] = b->ran[i] ? ms : -1.f;
    }
    return XSLAM_OK;
  }
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    ms_out[i] = -1.f;
    if (!b->ran[i]) continue;
    if (hipEventSynchronize(b->e1[i]) != hipSuccess) return XSLAM_ERR_HIP;
    if (hipEventElapsedTime(&ms_out[i], b->e0[i], b->e1[i]) != hipSuccess) return XSLAM_ERR_HIP;
  }
  return XSLAM_OK;
}

int32_t xslam_batch_last_index(xslam_batch b) { return b ? b->last_index : -1; }

int xslam_batch_destroy(xslam_batch b) {
  if (!b) return XSLAM_ERR_ARG;
  for (auto g : b->groups) delete g;   // (waits for the group's stream)
  for (size_t i = 0; i < b->e0.size(); ++i) {
    if (b->ran[i]) hipEventSynchronize(b->e1[i]);
    hipEventDestroy(b->e0[i]);
    hipEventDestroy(b->e1[i]);
  }
  delete b;
  return XSLAM_OK;
}

const char* xslam_last_error(xslam_ctx ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

int xslam_destroy(xslam_ctx ctx) {
  if (!ctx) return XSLAM_ERR_ARG;
  hipStreamSynchronize(ctx->stream);
  for (auto& e : ctx->timer.pool) hipEventDestroy(e);
  delete ctx->eng;
  delete ctx;
  return XSLAM_OK;
}

}  // extern "C"
