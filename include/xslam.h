/*
 * xslam.h -- C ABI of the MI355X CSFD dense-SLAM frame step.
 *
 * The library evaluates the KinectFusion-style frame step of X-SLAM (Peng et
 * al., ACM TOG 43(4) 2024; Sec. 4.1) -- surface measurement, projective
 * point-to-plane ICP, TSDF fusion and raycasting -- with every quantity carried
 * as a complex-step number x + i h x' (Sec. 3, eq. "csfd"), so that Im(f)/h is
 * the derivative of poses, maps and the TSDF with respect to chosen SLAM
 * parameters.  Products of two imaginary parts are dropped (Sec. 3, eqs.
 * "csfd_simplify_multiplication"/"csfd_simplify_division"), which makes the
 * arithmetic first-order dual numbers; second derivatives (Sec. 3, eqs.
 * "mc_taylor", "csfd_hessian") are carried as the i1*i2 parts of hyper-dual
 * numbers.  Many directions share one real part and run in one launch.
 *
 * Conventions
 *  - Every call returns int: 0 OK, < 0 error, > 0 warning.  Arguments are
 *    validated before anything is enqueued; no exception crosses the ABI.
 *  - Calls are asynchronous on the HIP stream given at creation, except those
 *    writing host memory (get, traj_err, step/track with pose_out), which
 *    synchronise that stream.  Errors of asynchronous kernels surface at the
 *    next synchronising call as XSLAM_ERR_HIP with text in xslam_last_error().
 *  - One host thread per context.
 *  - The caller owns all device memory: one workspace of
 *    xslam_workspace_bytes() bytes (256-byte aligned) passed to xslam_create;
 *    the context owns only its sub-allocation plan inside it.  Depth inputs are
 *    device pointers owned by the caller, read before the call's work ends.
 *  - World frame: origin at the volume centre, volume [-L/2, L/2]^3 with voxel
 *    centres at (i + 1/2) s - L/2.  Camera: x right, y down, z forward; pixel
 *    centres at integer coordinates.  Poses are camera-to-world, FP64,
 *    row-major 4x4.
 *  - A "component" of a scalar: 0 = real part, 1..D = the D first-order parts
 *    (direction d carries h_d times its derivative), D+1 .. D+P = the P
 *    second-order parts (pair (a,b) carries h_a h_b times the mixed derivative).
 *    Arrays of scalars cross the ABI as component planes:
 *    [re | tangent_0 .. tangent_{D-1} | second_0 .. second_{P-1}].
 */
#ifndef XSLAM_H
#define XSLAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xslam_ctx_s* xslam_ctx;

enum xslam_status {
  XSLAM_OK = 0,
  XSLAM_WARN_TRACK_LOST = 1,   /* pose kept (the ICP initial pose), fusion skipped */
  XSLAM_ERR_ARG = -1,
  XSLAM_ERR_WORKSPACE = -2,
  XSLAM_ERR_HIP = -3,
  XSLAM_ERR_STATE = -4,
  XSLAM_ERR_UNSUPPORTED = -5
};

/* arithmetic of the bulk of the frame step; the 6x6 solve, the SE(3)
 * exponential, pose composition and the trajectory error are always FP64 */
enum xslam_prec { XSLAM_C64 = 0 /* FP32 real + FP32 parts */, XSLAM_C128 = 1 /* FP64 */ };

/* perturbable parameters (Sec. 4.1: depth eq. "csfd_depth", pose eq. "lie") */
enum xslam_param {
  XSLAM_P_PHI_X = 0, XSLAM_P_PHI_Y, XSLAM_P_PHI_Z,   /* initial pose, rotation, left-multiplied  */
  XSLAM_P_RHO_X, XSLAM_P_RHO_Y, XSLAM_P_RHO_Z,       /* initial pose, translation, left-multiplied */
  XSLAM_P_TRUNC = 6,    /* truncation distance mu                          */
  XSLAM_P_WCAP = 7,     /* weight cap                                      */
  XSLAM_P_DGATE = 8,    /* ICP distance gate (hard gate: derivative 0)     */
  XSLAM_P_AGATE = 9,    /* ICP angle gate (hard gate: derivative 0)        */
  XSLAM_P_ICPW0 = 10,   /* ICP step relaxation of level 0, 1, 2 (10..12)   */
  XSLAM_P_FX = 13, XSLAM_P_FY = 14, XSLAM_P_CX = 15, XSLAM_P_CY = 16,
  XSLAM_P_DEPTH = 17,   /* caller supplies dD/dtheta per frame (depth_dot)   */
  XSLAM_P_COUNT = 18
};

/* one complex-step direction: parameter and step h (h > 0) */
typedef struct { int32_t param; double h; } xslam_dir;
/* one second-order pair: indices a <= b into the directions.  The set of
 * pairs must be every (a, b) with a <= b < Q for some Q <= D (the Hessian over
 * the first Q directions, listed in that row-major order). */
typedef struct { int32_t a, b; } xslam_pair;
typedef struct {
  int32_t n_dirs; const xslam_dir* dirs;
  int32_t n_pairs; const xslam_pair* pairs;
} xslam_perturbation;

typedef struct { int32_t width, height; double fx, fy, cx, cy; } xslam_camera;
/* dims must be multiples of 8 (8^3 bricks) */
typedef struct { int32_t dim[3]; double voxel; double trunc; double wcap; } xslam_volume;
typedef struct {
  int32_t iters[3];      /* per level, level 0 finest; levels run 2 -> 1 -> 0;
                            at most 25 passes in total                           */
  double dgate;          /* metres                                               */
  double agate_deg;      /* degrees                                              */
  double level_w[3];     /* step relaxation per level (1 = plain Gauss-Newton)   */
  double disc_delta;     /* depth discontinuity threshold of bilinear lookups (m)*/
  int32_t init;          /* 0: previous pose, 1: constant velocity (the previous
                            pose when either of the two previous frames was
                            lost), 2: network candidate judged against constant
                            velocity by one level-2 association pass: it is
                            used when its mean squared residual is lower and it
                            keeps >= 100 and >= 95% of the correspondences
                            (640 x 480 only; without an attached network it
                            behaves as 1)                                      */
  int32_t update;        /* pose update of a pass: 0 T <- exp(delta) T, the exact
                            SE(3) exponential (Sec. 4.1 eqs. lie, rotvector,
                            rotation_jacobi); 1 the small-angle matrix of eq.
                            icp_approx (rotation I + [phi]x, translation rho)
                            composed with T, its rotation then brought back to
                            orthonormal by two polar Newton steps -- the
                            original KinectFusion linearisation, kept as a
                            comparison form                                    */
  int32_t solver;        /* 0 Gauss-Newton (normal equations of the residual
                            linearised with the correspondences held fixed);
                            Newton (Sec. 4.1, the second-order ICP step): per
                            pass the gradient and Hessian of E = sum r^2 in the
                            increment from six hyper-dual directions and their
                            21 pairs (eq. csfd_hessian), with the pass's
                            correspondences held fixed (1) or differentiated
                            through the projective association (2);
                            delta = -H^-1 g when H passes the solver's pivot
                            test, else the Gauss-Newton step (counter slot 34
                            counts those passes).  Newton needs a perturbation
                            of no directions (XSLAM_ERR_ARG otherwise)         */
} xslam_icp;
/* The global model (Sec. 4): the TSDF volume of KinectFusion (Sec. 4.1), or
 * the surfel map of the PointFusion front end (Sec. 4.2: surfels with
 * position, normal, radius, confidence and time stamp; data association
 * through an index map rendered at 4 x 4 the image resolution, every surfel
 * of a pixel's block within the three gates updated with a Gaussian weight
 * of its distance times the measurement confidence exp(-gamma^2 / 0.72),
 * gamma the pixel's radial distance from the principal point over that of
 * the image corner; unassociated pixels appended as new surfels in pixel
 * order).  Tracking is the same ICP against the model maps, which the surfel
 * map renders as the nearest stable surfel per pixel. */
enum xslam_map { XSLAM_MAP_TSDF = 0, XSLAM_MAP_SURFEL = 1 };
typedef struct {
  double d_depth;        /* gate: |camera z of the surfel - measured z| (m)       */
  double d_norm_deg;     /* gate: angle between surfel and measured normal        */
  double d_dist;         /* gate: distance to the measured point (m)              */
  double sigma;          /* Gaussian weight exp(-d^2 / (2 sigma^2)) (m)           */
  double c_stable;       /* confidence a surfel needs to enter the model maps     */
  int32_t capacity;      /* maximum number of surfels (> 0); insertions past it
                            are dropped and counted (counter slot 36)             */
} xslam_surfel;
typedef struct {
  int32_t prec;          /* enum xslam_prec                                       */
  xslam_camera cam;      /* width, height multiples of 4                           */
  xslam_volume vol;
  xslam_icp icp;
  int32_t bilateral_radius;        /* 0 disables the filter                        */
  double bilateral_sigma_px, bilateral_sigma_m;
  double near_m;                   /* raycast near plane                           */
  int32_t max_frames;              /* capacity of the pose history                 */
  int32_t map;                     /* enum xslam_map: the global model              */
  xslam_surfel surfel;             /* surfel front end (map = XSLAM_MAP_SURFEL)     */
} xslam_config;

/* get/set fields */
enum xslam_field {
  XSLAM_F_POSE = 0,      /* current pose: [NC][16] double                                    */
  XSLAM_F_POSES = 1,     /* pose history: [frames][NC][16] double; set writes rows 0..n-1    */
  XSLAM_F_TSDF = 2,      /* F: [NC][N] in the context precision, N = dims product, x fastest */
  XSLAM_F_WEIGHT = 3,    /* W: [NC][N] (only the re and weight-cap parts can be nonzero)     */
  XSLAM_F_VMAP = 4,      /* model vertex map level 0 (world): [3][NC][H*W]                   */
  XSLAM_F_NMAP = 5,      /* model normal map level 0 (world): [3][NC][H*W]                   */
  XSLAM_F_ZMAP = 6,      /* model camera depth of the hits (real): [H*W]                     */
  XSLAM_F_MVALID = 7,    /* model validity: uint8 [H*W]                                      */
  XSLAM_F_MEAS_DEPTH = 8,/* filtered depth of levels 0,1,2 concatenated: [NC][n_l] per level */
  XSLAM_F_MEAS_V = 9,    /* measured vertex maps (camera), levels 0,1,2: [3][NC][n_l] each   */
  XSLAM_F_MEAS_N = 10,   /* measured normal maps (camera), levels 0,1,2                      */
  XSLAM_F_MEAS_VALID = 11,/* measured validity, uint8, levels 0,1,2                          */
  XSLAM_F_COUNTERS = 12, /* per frame int32[40]: 0 lost, 1 fused voxels, 2 raycast hits,
                            3 sum of ICP correspondences, 4 last-pass correspondences,
                            5..29 correspondences of every ICP pass, 30 bricks visited by
                            fusion, 31 raycast samples, 32 first ICP pass (1-based) whose
                            update norm |xi| fell below 1e-6 (0: none),
                            33 initialiser used (1 network, 0 constant velocity),
                            34 Newton passes that took the Gauss-Newton step,
                            surfel map: 1 surfel updates, 2 valid model pixels,
                            35 surfels inserted, 36 insertions dropped at the
                            capacity, 37 surfels in use;
                            38..39 reserved (0); set writes rows 0..n-1 (resume)            */
  XSLAM_F_PREV_POSE = 13,/* pose of the previous frame (ICP projection reference): [NC][16]  */
  XSLAM_F_FRAME = 14,    /* frame counter: int32                                             */
  /* surfel map (map = XSLAM_MAP_SURFEL; XSLAM_ERR_ARG otherwise), capacity C entries;
   * get copies all C, set writes the leading entries the buffer holds */
  XSLAM_F_SURF_V = 15,   /* positions (world): [3][NC][C] in the context precision          */
  XSLAM_F_SURF_N = 16,   /* normals: [3][NC][C]                                              */
  XSLAM_F_SURF_R = 17,   /* radii: [NC][C]                                                   */
  XSLAM_F_SURF_C = 18,   /* confidences: [NC][C]                                             */
  XSLAM_F_SURF_T = 19,   /* time stamps (frame index of the last update): int32 [C]          */
  XSLAM_F_SURF_COUNT = 20/* surfels in use: int32                                            */
};

/* number of components NC = 1 + D + P of a perturbation */
int32_t xslam_components(const xslam_perturbation* pert);

size_t xslam_workspace_bytes(const xslam_config* cfg, const xslam_perturbation* pert);

/* Create a context.  dev_workspace: device memory of at least
 * xslam_workspace_bytes(); stream: hipStream_t (NULL = default stream);
 * T0: initial camera pose (host, FP64 row-major 4x4); pose directions are
 * applied as exp(i h e_d) T0 (left multiplication).  The perturbation is
 * copied; the TSDF starts empty (F = 0, W = 0). */
int xslam_create(const xslam_config* cfg, const xslam_perturbation* pert, void* dev_workspace,
                 size_t bytes, void* stream, const double T0[16], xslam_ctx* out);

/* Surface measurement (Sec. 4.1 eq. "surface_measure"): promote the depth
 * (eq. "csfd_depth"; depth_dot holds one H*W plane per XSLAM_P_DEPTH
 * direction, in direction order, or NULL if there is none), bilateral filter,
 * pyramid, vertex and normal maps.  depth: device, float (C64) or double (C128). */
int xslam_measure(xslam_ctx ctx, const void* depth, const void* depth_dot);

/* Surface update (Sec. 4.1 "Surface Update"): fuse the last measured frame
 * into the TSDF at the current pose, or at `pose` (host FP64 4x4, zero
 * tangents) if not NULL.  depth != NULL measures it first. */
int xslam_integrate(xslam_ctx ctx, const void* depth, const void* depth_dot, const double* pose);

/* Surface prediction (Sec. 4.1 eq. "surface_prediction"): raycast the TSDF at
 * the current pose (or `pose`, host FP64 4x4) into the model maps (levels
 * 0..2).  vmap/nmap, if not NULL, receive copies of level 0 (device,
 * [3][NC][H*W] in the context precision). */
int xslam_raycast(xslam_ctx ctx, const double* pose, void* vmap, void* nmap);

/* Camera pose estimation (Sec. 4.1 eq. "icp"): measure `depth` (or, with
 * depth NULL, keep the maps measured last or set with xslam_set) and run the
 * multi-level ICP against the current model maps.  The result becomes the
 * current pose; pose_out (host, [NC][16]) if not NULL (synchronises). */
int xslam_track(xslam_ctx ctx, const void* depth, const void* depth_dot, double* pose_out);

/* Whole frame step: frame 0 fuses and raycasts at the initial pose; later
 * frames measure, track against the previous model maps, fuse (skipped when
 * tracking is lost) and raycast.  pose_out as in xslam_track.  The device
 * work of a tracked frame is captured once into a graph and replayed, except
 * on the legacy null stream (stream NULL at xslam_create), which cannot be
 * captured: there it is launched kernel by kernel (same results). */
int xslam_step(xslam_ctx ctx, const void* depth, const void* depth_dot, double* pose_out);

/* One association + normal-equation pass (no solve) of ICP level `level`
 * between the measured maps and the model maps of that level at the current
 * pose (projection reference: XSLAM_F_PREV_POSE).  sums_out (host): [NC][27]
 * doubles (21 upper-triangle entries of A row-major, then b), followed by
 * 2 doubles: correspondence count and sum of squared real residuals. */
int xslam_icp_pass(xslam_ctx ctx, int32_t level, double* sums_out);

/* The Newton objective of one ICP pass at level `level` (Sec. 4.1, the
 * second-order ICP step): E = sum of squared point-to-plane residuals between
 * the measured maps and the model maps of that level at the current pose
 * (projection reference: XSLAM_F_PREV_POSE), with its gradient and Hessian in
 * the left increment exp(delta) T.  through 0: the pass's correspondences
 * held fixed (the looked-up model point and normal are constants); through 1:
 * every residual differentiated through the projection, the bilinear model
 * lookup and its fractional weights (gates decided on real parts).  out
 * (host, 29 doubles): E, g[6], H (21, upper triangle row-major, order phi_x
 * phi_y phi_z rho_x rho_y rho_z), count.  Only for contexts with no
 * directions (XSLAM_ERR_UNSUPPORTED otherwise). */
int xslam_icp_energy(xslam_ctx ctx, int32_t level, int32_t through, double* out);

/* Camera relocalisation objective (Sec. 5.2): E(T_q) = sum over voxels of
 * (F_r - F_q)^2, where F_r is the context's TSDF (the reference volume M_r,
 * built by earlier frames or set with xslam_set) and F_q the same volume
 * after the last measured frame (the query depth, xslam_measure) is fused
 * into it at the candidate pose `pose` (host, FP64 row-major 4x4,
 * camera-to-world).  Only voxels the reference has observed (W_r > 0) and
 * that fusion would update contribute, each ((F_r - F_D) / (W_r + 1))^2 with
 * fusion's decisions and F_D; the volume, the current pose and the frame
 * state are left unchanged.  out (host, 29 doubles): E, its gradient g[6] and
 * Hessian H (21, upper triangle row-major) in the left increment
 * exp(delta) T_q, order phi_x phi_y phi_z rho_x rho_y rho_z (six hyper-dual
 * directions and their 21 pairs: the six complex-step and 21 bicomplex
 * evaluations of the surface update in one pass), then the number of
 * contributing voxels.  Synchronises.  Only for contexts with no directions
 * (XSLAM_ERR_UNSUPPORTED otherwise); XSLAM_ERR_STATE before any measured
 * frame; XSLAM_ERR_ARG for NULL or non-finite arguments. */
int xslam_reloc_energy(xslam_ctx ctx, const double pose[16], double* out);

/* Translational RMSE of the pose history against gt_poses (host, n x 16
 * FP64), no alignment; out (host): NC doubles (value and its parts).  FP64. */
int xslam_traj_err(xslam_ctx ctx, const double* gt_poses, int32_t n, double* out);

/* host <-> context state copies (host buffers; synchronising).  A checkpoint
 * that resumes a sequence bit for bit is the set of fields every later frame
 * reads: TSDF, WEIGHT, VMAP, NMAP, ZMAP, MVALID, POSE, PREV_POSE, POSES,
 * COUNTERS and FRAME, written back into a context created with the same
 * configuration and perturbation (brick flags and the level 1-2 model maps
 * are rebuilt from them); with the surfel map, the SURF_* fields and
 * SURF_COUNT take the place of TSDF and WEIGHT. */
int xslam_get(xslam_ctx ctx, int32_t field, void* dst, size_t bytes);
int xslam_set(xslam_ctx ctx, int32_t field, const void* src, size_t bytes);

/* Per-kernel timing with HIP events on the context stream (0 off, 1 on;
 * while on, tracked frames launch eagerly instead of through the graph);
 * xslam_kernel_times waits for the stream and writes accumulated
 * milliseconds and launch counts for 8 kernel classes: 0 measurement
 * (bilateral, pyramid, vertex/normal maps), 1 k_icp (association and
 * per-workgroup sums), 2 k_fuse, 3 k_raymarch, 4 other small kernels, 5
 * k_icp_finish (cross-workgroup sum, solve, pose update), 6 k_rayhit, 7
 * k_brick_cull. */
int xslam_set_timing(xslam_ctx ctx, int32_t on);
int xslam_kernel_times(xslam_ctx ctx, double ms_out[8], int64_t launches_out[8]);

/* ---- launch shapes and the autotuner ----------------------------------------
 * Launch shapes that do not change any result bit except the order of the
 * FP64 cross-block ICP sums (rounding level): the raycast tile (threads per
 * workgroup in x and y; x*y a multiple of 64 in [64, 256]), the ICP grid per
 * pyramid level (workgroups of 256 threads, 1..1200; 0 = one pixel per thread
 * up to 1200 workgroups) and the fusion grid (workgroups of one 8^3 brick each,
 * 64..4096, a grid-stride loop over the active-brick list).  Setting shapes
 * drops the captured frame graph (it is captured again on the next step).
 * Errors: XSLAM_ERR_ARG for a shape outside these limits. */
typedef struct {
  int32_t ray_tile[2];   /* raycast workgroup (x, y); default 16 x 16          */
  int32_t icp_blocks[3]; /* ICP workgroups at levels 0, 1, 2; 0 = default       */
  int32_t fuse_blocks;   /* fusion workgroups; default 4096                      */
  int32_t reserved[2];   /* 0                                                    */
} xslam_launch;

int xslam_set_launch(xslam_ctx ctx, const xslam_launch* shapes);
/* *active = 1 if tracked frames replay a captured graph (captured at the
 * first tracked step on a stream that can be captured), 0 if they launch
 * kernel by kernel (legacy null stream, per-kernel timing on, or before the
 * first tracked step).  Errors: XSLAM_ERR_ARG for a NULL active. */
int xslam_frame_graph(xslam_ctx ctx, int32_t* active);
/* the shapes in use (defaults resolved to numbers) */
int xslam_get_launch(xslam_ctx ctx, xslam_launch* out);
/* Time every candidate shape of the stages that can be re-run without
 * changing state, with HIP events (reps launches each, after one untimed
 * launch), and keep the fastest: the raycast tile (re-running the raycast of
 * the current pose rewrites the same model maps) and the ICP grid of each
 * level (association and sums only; the pose is not changed; the reps passes
 * are captured into a graph and replayed, so that short passes are not timed
 * at the host's launch rate; each candidate is timed in 3 rounds and a smaller
 * grid replaces a larger one only when 5% faster).  The fusion
 * grid changes the TSDF when run, so it is not timed here: time real steps
 * with different fuse_blocks instead (no result depends on it).  Requires a
 * measured frame and model maps (after xslam_step).  best (optional)
 * receives the shapes in use afterwards; ms_out (optional, 4 doubles) the
 * best mean times (ms) of raycast, ICP level 0, level 1 and level 2. */
int xslam_autotune(xslam_ctx ctx, int32_t reps, xslam_launch* best, double* ms_out);

/* ---- several independent sequences (multi-instance) -----------------------
 * A batch advances independent contexts (each its own sequence, volume,
 * image size and perturbation) by one frame each per call.  Every context's
 * frame step is enqueued on the stream it was created with; contexts created
 * on distinct streams run concurrently on the device, so small volumes and
 * the latency-bound ICP passes of one sequence overlap with the work of the
 * others.  Per context, HIP events around its frame give the frame's latency
 * on the device under that load.  The batch does not own the contexts: they
 * must outlive it.  Errors: XSLAM_ERR_ARG (NULL, n < 1, a context twice);
 * xslam_batch_step returns the first failing context's code, and its index
 * is in xslam_batch_last_index. */
typedef struct xslam_batch_s* xslam_batch;
int xslam_batch_create(const xslam_ctx* ctxs, int32_t n, xslam_batch* out);
/* The same batch advanced by grouped launches: contexts of one shape
 * (precision, directions, Hessian size) created on one stream form a group
 * (at most 32 per group, in context order) and are stepped together, one
 * launch per stage of the tracked frame for all of them; groups on different
 * streams overlap.  Each context contributes a descriptor (its own launch
 * arguments) and its own grid of work items (pixel tiles, bricks, ICP
 * workgroups); the grouped kernels' workgroups take the concatenated
 * (context, item) list in a fixed stride and run each item as the context's
 * own launch would, so every context's results equal its solo run bit for
 * bit.  The work of a group is captured into a graph and replayed until the
 * set of stepping contexts changes; a context's frame 0 runs its own step.
 * persist: workgroups per grouped launch, a multiple of 8 (0: one per work
 * item).  Requirements: the TSDF map, icp.solver 0, no network initialiser
 * attached, kernel timing off.  The raycast tile of a group is that of its
 * first context; launch shapes (xslam_set_launch) are read when a group's
 * plan is built, at its first grouped step and whenever the set of stepping
 * contexts changes.  The library
 * allocates the groups' descriptor tables (device memory, freed by
 * xslam_batch_destroy).  Latency (xslam_batch_latency) is that of the
 * context's group's step: from its first launch to its last.  Errors:
 * XSLAM_ERR_ARG (as above, a persist that is negative or not a multiple of 8,
 * contexts on different devices),
 * XSLAM_ERR_UNSUPPORTED (surfel map or Newton solver; the context's error
 * text names it), XSLAM_ERR_HIP. */
int xslam_batch_create_grouped(const xslam_ctx* ctxs, int32_t n, int32_t persist, xslam_batch* out);
/* depths[i] / depth_dots[i]: the frame of context i (device pointers, layout
 * as in xslam_step; depth_dots may be NULL); active (optional, n flags):
 * contexts with 0 are skipped (finished sequences). */
int xslam_batch_step(xslam_batch b, const void* const* depths, const void* const* depth_dots,
                     const int32_t* active);
/* waits for the last step of every context; ms_out[i] = device time from
 * the start to the end of context i's last frame step (-1 if it was skipped) */
int xslam_batch_latency(xslam_batch b, float* ms_out);
int32_t xslam_batch_last_index(xslam_batch b);
int xslam_batch_destroy(xslam_batch b);

/* ---- learned ICP initialiser (a systems form beyond the paper) -------------
 * A CNN proposes the ICP initial pose increment from coarse maps: input
 * 5 x 60 x 80 FP32 (current depth at pyramid level 3; raycast depth and raycast
 * normal (x, y, z) of the previous frame in its camera frame; invalid pixels
 * 0), four 3x3 stride-2 convolutions with ReLU (5->16->32->64->128), global
 * average pool, 128->64 (ReLU)->6 = (phi, rho), the right increment of the
 * previous camera pose.  bf16 MFMA convolutions with FP32 accumulation; FP32
 * master weights and Adam (beta 0.9, 0.999, eps 1e-8).  Loss: mean over the
 * batch of |100 (xi_hat - xi)|^2.  Parameters are one FP32 vector in the order
 * conv0 W (Co,Ci,3,3), b, conv1 W, b, conv2 W, b, conv3 W, b, fc1 W (64,128),
 * b, fc2 W (6,64), b.  The caller owns the workspace; calls are asynchronous
 * on the given stream except get/set and train_step with loss_out. */
typedef struct xslam_cnn_s* xslam_cnn;
int32_t xslam_cnn_param_count(void);
size_t xslam_cnn_workspace_bytes(int32_t max_batch);
int xslam_cnn_create(void* dev_workspace, size_t bytes, void* stream, int32_t max_batch, xslam_cnn* out);
int xslam_cnn_set_weights(xslam_cnn cnn, const float* host, size_t n);   /* also resets Adam */
int xslam_cnn_get_weights(xslam_cnn cnn, float* host, size_t n);
int xslam_cnn_get_grads(xslam_cnn cnn, float* host, size_t n);           /* of the last train step */
/* x_dev: n x 5 x 60 x 80 FP32 device; xi_dev: n x 6 FP32 device */
int xslam_cnn_forward(xslam_cnn cnn, const float* x_dev, int32_t n, float* xi_dev);
/* xslam_cnn_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, with the forward activations in a fixed device
 * array of the library (about 3.9 MB, one per GPU, held until the process
 * ends) instead of the handle's workspace, so any handle (also one created
 * with max_batch 1) serves batches of up to 32.  n > 32: XSLAM_ERR_WORKSPACE
 * with the reason in xslam_cnn_last_error.  Nothing is allocated.  Every call
 * on one GPU shares that array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller. */
int xslam_cnn_forward_noalloc(xslam_cnn cnn, const float* x_dev, int32_t n, float* xi_dev);
/* one Adam step on a batch; label_dev n x 6 FP32 device; loss_out host or NULL */
int xslam_cnn_train_step(xslam_cnn cnn, const float* x_dev, const float* label_dev, int32_t n, float lr,
                         float* loss_out);
const char* xslam_cnn_last_error(xslam_cnn cnn);
int xslam_cnn_destroy(xslam_cnn cnn);

/* Attach a network to a context for icp.init 2; NULL detaches.  The network
 * must have been created on the context's stream (XSLAM_ERR_ARG otherwise):
 * its forward pass then runs in the context's stream order and inside the
 * context's captured frame graph.  Each tracked frame then builds the input from its measured
 * depth and the previous model maps, proposes T_{k-1} exp(xi), and keeps the
 * candidate (network or constant velocity) with the lower mean squared
 * point-to-plane residual of one level-2 association pass; the network's only
 * with at least 100 correspondences.  The network output is real: it carries
 * no derivative. */
int xslam_ctx_set_cnn(xslam_ctx ctx, xslam_cnn cnn);
/* Network input parts of the current state (training data): depth_dev
 * 60 x 80 FP32 (the last measured frame at level 3), model_dev 4 x 60 x 80
 * FP32 (the last raycast: hit depth and normal in the camera frame of the
 * current pose).  Device pointers; synchronises. */
int xslam_cnn_parts(xslam_ctx ctx, float* depth_dev, float* model_dev);

int xslam_sync(xslam_ctx ctx);
const char* xslam_last_error(xslam_ctx ctx);
int xslam_destroy(xslam_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* XSLAM_H */
