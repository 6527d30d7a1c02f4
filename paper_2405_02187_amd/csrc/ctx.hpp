// Host-side context of the C ABI.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>
#include "../../include/xslam.h"

namespace xs {

// Event pair of the launch in progress (timing mode; null otherwise).  With
// events the kernel goes through hipExtLaunchKernelGGL, whose dispatch stamps
// them with the kernel's own start and end.
inline thread_local hipEvent_t tl_ev0 = nullptr;
inline thread_local hipEvent_t tl_ev1 = nullptr;
#define XS_LAUNCH(kernel, grid, block, shmem, stream, ...)                                                   \
  do {                                                                                                      \
    if (::xs::tl_ev0)                                                                                       \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ::xs::tl_ev0, ::xs::tl_ev1, 0, __VA_ARGS__); \
    else                                                                                                    \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                                  \
  } while (0)

// Contexts per group of a grouped batch, and the multiple a grouped launch's
// workgroup count keeps (the XCD count: an item stays on the XCD its solo
// launch would give it).
constexpr int kGroupMax = 32;
constexpr int kGroupAlign = 8;

// Several contexts of one shape stepped by grouped launches (group.hpp).
// step: one frame of each member with active[m] != 0 (member order);
// failed_member: the member whose check failed after a non-zero return.
struct GroupBase {
  virtual ~GroupBase() {}
  virtual int step(const void* const* depths, const void* const* ddots, const int32_t* active) = 0;
  virtual int failed_member() const = 0;
  // device time of the group's last step (ms), -1 if it did nothing
  virtual float last_ms() = 0;
  virtual bool ran(int member) const = 0;
};

struct EngineBase {
  virtual ~EngineBase() {}
  // equal for engines of one (precision, directions, Hessian) shape
  virtual int shape_key() const = 0;
  // a group runner for n engines of this engine's shape (es[0] is this one),
  // launching on stream; persist: workgroups of a grouped launch (0: one per item)
  virtual GroupBase* new_group(EngineBase* const* es, int n, hipStream_t stream, int persist) = 0;
  virtual int measure(const void* depth, const void* ddot) = 0;
  virtual int integrate(const double* pose) = 0;
  virtual int raycast(const double* pose, void* vmap, void* nmap) = 0;
  virtual int track() = 0;
  virtual int step(const void* depth, const void* ddot) = 0;
  virtual int icp_pass(int level, double* out) = 0;
  virtual int icp_energy(int level, int through, double* out) = 0;
  virtual int reloc_energy(const double* pose, double* out) = 0;
  virtual int traj_err(const double* gt, int n, double* out) = 0;
  virtual int get(int field, void* dst, size_t bytes) = 0;
  virtual int set(int field, const void* src, size_t bytes) = 0;
  virtual int current_pose(double* out) = 0;
  // lost flag of the frame just stepped (stepped) or of the frame tracked
  // stage by stage, whose counter row is the current frame index
  virtual int frame_lost(int* lost, bool stepped) = 0;
  virtual int set_cnn(xslam_cnn cnn) = 0;
  virtual int cnn_parts(float* depth, float* model) = 0;
  virtual int set_launch(const xslam_launch& l) = 0;
  virtual int get_launch(xslam_launch* l) = 0;
  virtual bool frame_graph() const = 0;
  virtual int autotune(int reps, double* ms_out) = 0;
};

struct Timer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  static constexpr int kClasses = 8;
  double ms[kClasses] = {};
  int64_t launches[kClasses] = {};
};

}  // namespace xs

struct xslam_ctx_s {
  xslam_config cfg;
  std::vector<xslam_dir> dirs;
  std::vector<xslam_pair> pairs;
  int D = 0, Q = 0, NC = 1;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  xs::EngineBase* eng = nullptr;
  xs::Timer timer;
  int device = 0;
};
