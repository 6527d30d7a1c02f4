// Grouped launches: one grid runs a frame-step stage for several independent
// sequences (instances) of the same (precision, directions, Hessian) shape.
// Each instance brings a descriptor -- the arguments its own launch of the
// stage would take -- and a grid of work items (its pixel tiles, bricks or ICP
// workgroups).  The grouped kernel runs the stage's body on each item of the
// concatenated (instance, item) list exactly as the instance's own launch
// would, so every instance's results equal those of its solo run bit for bit:
// one workgroup per item (k_group_once), or a persistent grid whose
// workgroups take the list in a fixed stride (k_group).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "ctx.hpp"
#include "kernels.hpp"

namespace xs {

// first[i]: the instance's first item in the concatenated list, a multiple of
// the XCD count, so that an item's XCD is the one its solo launch would give
// it and the bodies' own XCD remaps keep their meaning.
static_assert(kGroupAlign == kXcds, "grouped grids keep the XCD of every item");

// (the item map travels by value in the kernel arguments)
struct GroupMap {
  int n, total;
  int first[kGroupMax + 1];
  int gx[kGroupMax], gy[kGroupMax];
};

template <class A>
__global__ __launch_bounds__(A::kThreads) void k_group(const A* __restrict__ desc, GroupMap m) {
  for (int w = blockIdx.x; w < m.total; w += gridDim.x) {
    int i = 0;
    while (i + 1 < m.n && m.first[i + 1] <= w) ++i;
    const int local = w - m.first[i], gx = m.gx[i], gy = m.gy[i];
    if (local < gx * gy) desc[i].run(VB{local % gx, local / gx, gx, gy});
    if (w + int(gridDim.x) < m.total) __syncthreads();   // the next item reuses the LDS
  }
}

// Descriptor pointers are stated to address global memory (PtrGlobal), as
// the solo launches' kernel arguments are; the nested argument structs are
// copied with their pointers so stated.
constexpr PtrGlobal kG{};
template <typename T, int D, int Q>
__device__ __forceinline__ TrackBegin<T, D, Q> as_global(const TrackBegin<T, D, Q>& a) {
  TrackBegin<T, D, Q> r = a;
  r.Pcur = kG(a.Pcur); r.Pprev = kG(a.Pprev); r.Pprev2 = kG(a.Pprev2); r.Pinit = kG(a.Pinit);
  r.Kcur = kG(a.Kcur); r.Kprev = kG(a.Kprev); r.lost = kG(a.lost); r.counter_base = kG(a.counter_base);
  r.frame = kG(a.frame);
  return r;
}
template <typename T, int D, int Q>
__device__ __forceinline__ IcpArgs<T, D, Q> as_global(const IcpArgs<T, D, Q>& a) {
  IcpArgs<T, D, Q> r = a;
  r.V = kG(a.V); r.N = kG(a.N); r.valid = kG(a.valid);
  r.Vm = kG(a.Vm); r.Nm = kG(a.Nm); r.Zm = kG(a.Zm); r.validm = kG(a.validm);
  r.Kcur = kG(a.Kcur); r.Kprev = kG(a.Kprev); r.Pcur = kG(a.Pcur);
  r.partials = kG(a.partials); r.lost = kG(a.lost); r.counters = kG(a.counters); r.frame = kG(a.frame);
  r.sums_out = kG(a.sums_out);
  return r;
}
template <typename T, int D, int Q>
__device__ __forceinline__ PostTrack<T, D, Q> as_global(const PostTrack<T, D, Q>& a) {
  PostTrack<T, D, Q> r = a;
  r.Pcur = kG(a.Pcur); r.Pinit = kG(a.Pinit); r.Kcur = kG(a.Kcur); r.lost = kG(a.lost);
  r.history = kG(a.history); r.frame = kG(a.frame); r.count = kG(a.count);
  return r;
}
template <typename T, int D, int Q>
__device__ __forceinline__ MapsOut<T, D, Q> as_global(const MapsOut<T, D, Q>& a) {
  MapsOut<T, D, Q> r;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    r.V[l] = kG(a.V[l]); r.N[l] = kG(a.N[l]); r.Z[l] = kG(a.Z[l]); r.valid[l] = kG(a.valid[l]);
  }
  return r;
}

// One workgroup per item (the grid covers the list): the same without the
// loop, whose live state across items costs the larger bodies registers
// (the ICP pass: 236 against 186 VGPRs)
template <class A>
__global__ __launch_bounds__(A::kThreads) void k_group_once(const A* __restrict__ desc, GroupMap m) {
  const int w = blockIdx.x;
  int i = 0;
  while (i + 1 < m.n && m.first[i + 1] <= w) ++i;
  i = __builtin_amdgcn_readfirstlane(i);
  const int local = w - m.first[i], gx = m.gx[i], gy = m.gy[i];
  if (local < gx * gy) desc[i].run(VB{local % gx, local / gx, gx, gy});
}

// Stage descriptors: the arguments of the solo launch and the body it runs.
template <typename T, int D, int Q>
struct GBilateral {
  static constexpr int kThreads = 256;
  KParams<T, D, Q> kp;
  const T* depth; const T* ddot; T* Dout; double* Dhi;
  TrackBegin<T, D, Q> tb;
  __device__ __forceinline__ void run(const VB& vb) const { 
    const TrackBegin<T, D, Q> t = as_global(tb);
    bilateral_body<T, D, Q>(vb, kp, kG(depth), kG(ddot), kG(Dout), kG(Dhi), t);
  }
};

template <typename T, int D, int Q>
struct GPyrdown {
  static constexpr int kThreads = 256;
  KParams<T, D, Q> kp;
  const T* Din; int Wi, Hi; T* Dout; const double* Dhi_in; double* Dhi_out;
  __device__ __forceinline__ void run(const VB& vb) const {
    pyrdown_body<T, D, Q>(vb, kp, kG(Din), Wi, Hi, kG(Dout), kG(Dhi_in), kG(Dhi_out));
  }
};

template <typename T, int D, int Q>
struct GVertexNormal {
  static constexpr int kThreads = 256;
  KParams<T, D, Q> kp;
  VNLevels<T> lv;
  __device__ __forceinline__ void run(const VB& vb) const { vertex_normal_body<T, D, Q>(vb, kp, lv, kG); }
};

template <typename T, int D, int Q>
struct GIcp {
  static constexpr int kThreads = kIcpThreads;
  KParams<T, D, Q> kp;
  IcpArgs<T, D, Q> g;
  __device__ __forceinline__ void run(const VB& vb) const { 
    const IcpArgs<T, D, Q> a = as_global(g);
    icp_body<T, D, Q>(vb, kp, a);
  }
};

template <typename T, int D, int Q>
struct GIcpFinish {
  static constexpr int kThreads = kFinishThreads<T, D, Q>;
  IcpArgs<T, D, Q> g;
  int nblocks;
  __device__ __forceinline__ void run(const VB& vb) const { 
    const IcpArgs<T, D, Q> a = as_global(g);
    icp_finish_body<T, D, Q>(vb, a, nblocks);
  }
};

template <typename T, int D, int Q>
struct GTileZmax {
  static constexpr int kThreads = 256;
  const T* D0; int W, H; T* tmax; T* cmax;
  PostTrack<T, D, Q> post;
  __device__ __forceinline__ void run(const VB& vb) const { 
    const PostTrack<T, D, Q> p = as_global(post);
    tile_zmax_body<T, D, Q>(vb, kG(D0), W, H, kG(tmax), kG(cmax), p);
  }
};

template <typename T, int D, int Q>
struct GBrickCull {
  static constexpr int kThreads = 256;
  KParams<T, D, Q> kp;
  const KPose<T, D, Q>* Kk; const T* tmax; const T* cmax;
  int nbrick; int* list; int* count; const int* lost;
  __device__ __forceinline__ void run(const VB& vb) const {
    brick_cull_body<T, D, Q>(vb, kp, kG(Kk), kG(tmax), kG(cmax), nbrick, kG(list), kG(count), kG(lost));
  }
};

template <typename T, int D, int Q>
struct GFuse {
  static constexpr int kThreads = kBrickVox;
  KParams<T, D, Q> kp;
  const KPose<T, D, Q>* Kk; const T* Df; typename Vec2<T>::type* rec; T* Ftan; T* Wtan;
  const int* lost; int64_t nvox; const int* list; const int* count; int* block_counts;
  __device__ __forceinline__ void run(const VB& vb) const {
    fuse_body<T, D, Q>(vb, kp, kG(Kk), kG(Df), kG(rec), kG(Ftan), kG(Wtan), kG(lost), nvox, kG(list), kG(count),
                       kG(block_counts));
  }
};

template <typename T>
struct GBrickFlags {
  static constexpr int kThreads = kBrickVox;
  const typename Vec2<T>::type* rec; uint8_t* flags; const int* list; const int* count; int nbrick;
  const int* fcounts; int nf; int32_t* counter_base; const int* frame; int max_frames;
  __device__ __forceinline__ void run(const VB& vb) const {
    brick_flags_body<T>(vb, kG(rec), kG(flags), kG(list), kG(count), nbrick, kG(fcounts), nf, kG(counter_base),
                        kG(frame), max_frames);
  }
};

template <typename T>
struct GBrickApron {
  static constexpr int kThreads = 256;
  uint8_t* flags; int nbx, nby, nbz;
  __device__ __forceinline__ void run(const VB& vb) const { brick_apron_body<T>(vb, kG(flags), nbx, nby, nbz); }
};

template <typename T, int D, int Q>
struct GRaymarch {
  static constexpr int kThreads = 256;
  KParams<T, D, Q> kp;
  const KPose<T, D, Q>* Kk; const typename Vec2<T>::type* rec; const uint8_t* flags;
  typename Vec2<T>::type* bracket; int* block_samples;
  __device__ __forceinline__ void run(const VB& vb) const {
    raymarch_body<T, D, Q>(vb, kp, kG(Kk), kG(rec), kG(flags), kG(bracket), kG(block_samples));
  }
};

template <typename T, int D, int Q>
struct GRayhit {
  static constexpr int kThreads = 256;
  KParams<T, D, Q> kp;
  const KPose<T, D, Q>* Kk; const typename Vec2<T>::type* rec; const T* Ftan; int64_t nvox;
  const typename Vec2<T>::type* bracket; MapsOut<T, D, Q> out; int* block_hits;
  __device__ __forceinline__ void run(const VB& vb) const {
    const MapsOut<T, D, Q> o = as_global(out);
    rayhit_body<T, D, Q>(vb, kp, kG(Kk), kG(rec), kG(Ftan), nvox, kG(bracket), o, kG(block_hits));
  }
};

template <typename T>
struct GSumCounts {
  static constexpr int kThreads = 1024;
  const int* a; int n; const int* b; int nb; int32_t* counter_base; const int* frame; int max_frames;
  int slot_a, slot_b; const int* extra; int slot_extra; int* advance;
  __device__ __forceinline__ void run(const VB& vb) const {
    sum_counts_body<T>(vb, kG(a), n, kG(b), nb, kG(counter_base), kG(frame), max_frames, slot_a, slot_b, kG(extra),
                       slot_extra, kG(advance));
  }
};

// Input copies of a group's frame: entry e copies bytes[e] (a multiple of 16)
// from src[e] to dst[e] (both 16-byte aligned); blockIdx.y is the entry.
constexpr int kGroupCopyMax = 2 * kGroupMax;
struct CopyMap {
  int n;
  const void* src[kGroupCopyMax];
  void* dst[kGroupCopyMax];
  int64_t bytes[kGroupCopyMax];
};

template <typename T>
__global__ __launch_bounds__(256) void k_group_copy(CopyMap m) {
  const int e = blockIdx.y;
  const uint4* s = static_cast<const uint4*>(m.src[e]);
  uint4* d = static_cast<uint4*>(m.dst[e]);
  const int64_t n = m.bytes[e] >> 4;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) d[i] = s[i];
}

}  // namespace xs
