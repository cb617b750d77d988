/*
 * seb.h -- C ABI of the MI355X (gfx950) SE(2)-grid traversability library.
 *
 * Method: SEB-Naver (arXiv 2503.02412).  For every state (x, y, yaw) of a
 * robot-centric height map the library gathers the terrain under the
 * yaw-rotated vehicle footprint, fits the terrain plane, recovers the pose the
 * terrain imposes (Sec. III, Eq. 1-3: height z, and the body axes from the
 * plane normal z_b, reported as Z-X-Y roll and pitch) and scores the risk of
 * Algorithm 1 (Sec. V-B: curvature early-out, tilt early-out, weighted sum).
 * The map is robot-centric and moves with the robot (Sec. V-A, Eq. 4).
 *
 * Conventions shared by every entry point:
 *   - Heights: float32, row-major [H][W] with row stride `ld` (elements),
 *     NaN or +-Inf = unknown cell.  Finite heights must satisfy |h| < 2^60.
 *     Cell (ix, iy) is centred at map-local metres ((ix+0.5) res, (iy+0.5) res).
 *   - Yaw bins: theta_k = 2 pi k / K, k = 0 .. K-1.
 *   - Outputs (seb_out): five device arrays laid out [K][H][W] (yaw-major
 *     planes of H rows of W cells, dense).  Units: metres / radians.
 *   - All array pointers are DEVICE pointers owned by the caller; they must
 *     stay valid until the work queued on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls only enqueue work: they never synchronise, never print, and
 *     allocate device memory only in the *_create functions.
 *   - Return value: SEB_OK (0) or a negative seb_status.  Argument errors are
 *     detected on the host before anything is launched; seb_last_error()
 *     returns a thread-local message describing the most recent failure.
 *     Asynchronous device faults surface at the caller's next synchronisation.
 *   - A seb_ctx / seb_window may be used by one stream at a time.
 */
#ifndef SEB_H
#define SEB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SEB_OK = 0,
    SEB_ERR_INVALID = -1,      /* bad argument or configuration             */
    SEB_ERR_HIP = -2,          /* a HIP runtime call or launch failed       */
    SEB_ERR_ALLOC = -3,        /* device or host allocation failed          */
    SEB_ERR_UNSUPPORTED = -4,  /* valid, but outside what the kernels cover */
    SEB_ERR_IO = -5            /* file could not be read or written         */
} seb_status;

/* Status byte of each state. */
enum {
    SEB_ST_VALID = 1,       /* plane fitted; 0 = UNKNOWN (too few / collinear samples) */
    SEB_ST_CURV = 2,        /* Alg. 1 curvature early-out: kappa > kappa_max           */
    SEB_ST_TILT = 4,        /* Alg. 1 tilt early-out: phi_x > phi_x_max or phi_y > ... */
    SEB_ST_DEGEN = 8,       /* near-degenerate footprint (few or nearly collinear)     */
    SEB_ST_TRAV = 16,       /* traversable: valid and risk <= risk_max                 */
    SEB_ST_SURROGATE = 32   /* produced by the learned surrogate, not the plain fit    */
};

/* Assessment parameters.  Lengths in metres, angles in radians.  The names
 * follow Algorithm 1 (Sec. V-B): kappa_max, phi_x_max, phi_y_max and the risk
 * weights w_r = (w_kappa, w_phi_x, w_phi_y); risk_max is r_max of the safety
 * constraint (Sec. VI-B).  The paper gives phi_x_max = phi_y_max = 0.52 rad
 * (Sec. VII-B) and leaves the others open. */
typedef struct seb_config {
    int32_t width, height;       /* W (x, columns) and H (y, rows) cells          */
    double resolution;           /* metres per cell                               */
    int32_t n_yaw;               /* K                                             */
    double fp_length, fp_width;  /* footprint extent along body x / body y        */
    int32_t fp_nl, fp_nw;        /* body-frame midpoint sample grid               */
    int32_t fp_shape;            /* 0 rectangle, 1 inscribed ellipse              */
    double kappa_max, phi_x_max, phi_y_max;
    double w_kappa, w_phi_x, w_phi_y, risk_max;
    int32_t min_valid;           /* >= 3 samples needed for a fit                 */
    int32_t precision;           /* 0 FP32; 1 FP32 + FP64 for near-degenerate    */
    int32_t fit;                 /* 0 least-squares plane; 1 principal-component
                                    plane of Algorithm 1 (minimum eigenvector of
                                    the footprint covariance, solved in FP64)     */
} seb_config;

/* Output arrays, each [K][H][W] on the device.  z and the angles are NaN for
 * UNKNOWN states, whose risk is 1. */
typedef struct seb_out {
    float* z;       /* terrain-imposed height at the state (plane at the cell centre) */
    float* roll;    /* Z-X-Y roll, > 0 left side up                                 */
    float* pitch;   /* Z-X-Y pitch, > 0 nose down                                   */
    float* risk;    /* Algorithm 1 risk in [0, 1]; 1 = explicit obstacle            */
    uint8_t* status;/* SEB_ST_* bits                                                */
} seb_out;

typedef struct seb_ctx seb_ctx;
typedef struct seb_window seb_window;

/* ---------------------------------------------------------------- context */

/* Check a configuration on the host only (no device use).  Returns SEB_OK,
 * SEB_ERR_INVALID (malformed) or SEB_ERR_UNSUPPORTED (footprint reach or
 * sample grid beyond the kernels' limits). */
int seb_validate_config(const seb_config* cfg);

/* Build the FP64 footprint/yaw table for `cfg` on the host and upload it to
 * the current HIP device: for every yaw bin theta_k = 2 pi k / K of the SE(2)
 * grid and every sample of the footprint of Sec. V-B (the vehicle's extent
 * under the yaw-rotated body frame of Sec. III, Eq. 1-3), the sample's map
 * offset split into an integer cell and bilinear weights.  *out receives the
 * new context (library-owned; release with seb_destroy).  Errors:
 * SEB_ERR_INVALID, SEB_ERR_UNSUPPORTED, SEB_ERR_ALLOC, SEB_ERR_HIP. */
int seb_create(const seb_config* cfg, seb_ctx** out);

/* Release a context and its device table.  NULL is ignored.  The caller must
 * ensure no queued work still uses it. */
void seb_destroy(seb_ctx* ctx);

/* ------------------------------------------------------ full assessment */

/* Assess every yaw bin of the states in the rectangle [x0, x0+nx) x
 * [y0, y0+ny) of the map `height` (device, [H][W] with row stride ld >= W),
 * writing out->*[k][iy][ix] for those states only.  Footprint samples that
 * fall outside the map or on unknown cells are dropped (Alg. 1 runs on the
 * valid ones).  nx == 0 or ny == 0 is a no-op.  The rectangle must lie inside
 * the map.  Defined by Sec. V-B, Algorithm 1 with Eq. 1-3 of Sec. III. */
int seb_assess_se2(seb_ctx* ctx, const float* height, int64_t ld, int32_t x0, int32_t y0,
                   int32_t nx, int32_t ny, const seb_out* out, void* stream);

/* ------------------------------------------------- rolling maintenance */

/* Geometry of one window move (host only, pure integer arithmetic). */
typedef struct seb_window_plan {
    int64_t old_origin_x, old_origin_y;   /* world cell of logical cell (0, 0)       */
    int64_t new_origin_x, new_origin_y;   /* Eq. 4: floor(p / res) - (W/2, H/2)      */
    int32_t full_reset;                   /* shift >= window size: everything new    */
    int32_t exposed_rows;                 /* |dy| whole rows (W cells each)          */
    int32_t exposed_cols;                 /* |dx| columns over the other H-|dy| rows */
    int64_t n_cells_exposed;              /* cells new_cells must provide            */
    int32_t n_rects;                      /* disjoint state rectangles recomputed    */
    int32_t rects[8][4];                  /* x0, y0, nx, ny in new logical coords    */
    int64_t n_states;                     /* states recomputed (all yaw bins)        */
} seb_window_plan;

/* Create a rolling window over caller-owned ring storage: `height_ring`
 * ([H][W], row stride ld) and `out_ring` (seb_out, [K][H][W]).  World cell
 * (gx, gy) of the window lives at ring position (gx mod W, gy mod H) in both.
 * The window starts at the robot position (x, y) metres with every cell
 * unknown; call seb_window_reset to load heights.  Errors: SEB_ERR_INVALID,
 * SEB_ERR_ALLOC. */
int seb_window_create(seb_ctx* ctx, float* height_ring, int64_t ld, const seb_out* out_ring,
                      double x, double y, seb_window** out);
void seb_window_destroy(seb_window* w);

/* Origin (world cell of logical (0, 0)) and ring offset (origin mod size). */
int seb_window_origin(const seb_window* w, int64_t* origin_x, int64_t* origin_y,
                      int32_t* ring_x, int32_t* ring_y);

/* Place the window at robot position (x, y) (Eq. 4), copy the logical map
 * `heights` (device [H][W], row stride ld; NULL = all unknown) into the ring
 * and assess every state. */
int seb_window_reset(seb_window* w, double x, double y, const float* heights, int64_t ld,
                     void* stream);

/* Host-only geometry of moving the window to robot position (x, y): the new
 * origin by Eq. 4, the exposed strips and the rectangles of states whose
 * footprint reaches a changed cell (new cells, or cells that left the window
 * and are unknown from now on).  Does not modify the window. */
int seb_window_plan_move(const seb_window* w, double x, double y, seb_window_plan* plan);

/* The same geometry without a window or a device: for a window of `cfg`
 * whose logical cell (0, 0) is world cell (origin_x, origin_y), moving the
 * robot to (x, y).  Host only. */
int seb_plan_window_move(const seb_config* cfg, int64_t origin_x, int64_t origin_y, double x,
                         double y, seb_window_plan* plan);

/* Move the window to robot position (x, y) (Sec. V-A: Eq. 4, then cells no
 * longer in the map become unknown).  `new_cells` (device, may be NULL = all
 * unknown) holds the heights of the newly exposed cells in the order of
 * seb_window_plan: first the exposed rows (increasing logical y, each W cells
 * of increasing x), then the exposed columns (for each remaining row in
 * increasing y, the |dx| cells in increasing x).  Then re-assesses exactly the
 * plan's rectangles; the result equals a full seb_assess_se2 of the new window
 * bit for bit.  *n_states_recomputed (host, may be NULL) receives the plan's
 * n_states without synchronising. */
int seb_update_window(seb_window* w, double x, double y, const float* new_cells, void* stream,
                      int64_t* n_states_recomputed);

/* ------------------------------------------------- learned surrogate */

/* A small network that maps the terrain around a cell plus the yaw to the
 * assessment's outputs (Sec. III Eq. 1-3, Sec. V-B Alg. 1).  Learned
 * traversability models are discussed in Sec. II, together with their model
 * uncertainty -- hence the plain-method fallback of seb_surrogate_infer.
 * Input of cell (cy, cx): three 24 x 24 channels over cells
 * (cy-12+i, cx-12+j): x-slope and y-slope (height differences to the next
 * cell / resolution, 0 unless both cells are known) and a known flag.
 * Layers: conv 3->16 (4x4, stride 2), conv 16->32 (3x3, stride 2), fc
 * 800 + (sin yaw, cos yaw) -> 128 -> 64 -> 4, ReLU between layers; bf16
 * weights and activations, fp32 accumulation.  Outputs (dz/0.05 m,
 * roll/0.5 rad, pitch/0.5 rad, risk) with dz = z - h_ref, h_ref being the
 * cell's own height when it is known, else the mean of its known in-map
 * 8-neighbours (a cell with neither has no network answer).
 * Parameters: float32 vector of seb_net_param_count() values, in the order
 * W1[16][3][4][4] b1[16] W2[32][16][3][3] b2[32] W3[128][800] Wy[128][2]
 * b3[128] W4[64][128] b4[64] W5[4][64] b5[4]; W3's 800 inputs are ordered
 * (row a, column b, channel) of conv2's 5 x 5 x 32 output. */
typedef struct seb_net seb_net;

/* A batch of training (or forward) samples drawn from a set of maps. */
typedef struct seb_train_batch {
    const float* maps;           /* device [n_maps][map_h][map_w] heights, NaN = unknown */
    int32_t n_maps, map_h, map_w;
    double resolution;
    int32_t n_yaw;               /* K of the labels; yaw k means theta = 2 pi k / K   */
    const float* label_z;        /* device [n_maps][K][map_h][map_w] plain-method     */
    const float* label_roll;     /* outputs for the maps (training only; may be NULL  */
    const float* label_pitch;    /* for seb_net_forward)                               */
    const float* label_risk;
    const int32_t* samples;      /* device [batch][4]: map, cy, cx, k                  */
    int32_t batch;               /* multiple of 32, <= the net's max_batch             */
} seb_train_batch;

int64_t seb_net_param_count(void);

/* Create a network with counter-based random initial weights (He-uniform
 * from splitmix64(seed, index)), zero biases and Adam state, and a training
 * workspace for batches up to max_batch (multiple of 32, <= 65536).
 * Synchronises the device.  Errors: SEB_ERR_INVALID, SEB_ERR_ALLOC, SEB_ERR_HIP. */
int seb_net_create(uint64_t seed, int32_t max_batch, seb_net** out);
void seb_net_destroy(seb_net* net);

/* Copy the float32 parameter vector to / from host memory (synchronous).
 * Setting parameters resets the Adam state. */
int seb_net_get_params(const seb_net* net, float* host_params);
int seb_net_set_params(seb_net* net, const float* host_params);

/* Checkpoint: parameters, Adam moments and step in one file ("SEBNET01",
 * int64 count, int64 step, then three float32 vectors).  Synchronous.
 * Errors: SEB_ERR_IO for unreadable / malformed files. */
int seb_net_save(const seb_net* net, const char* path);
int seb_net_load(seb_net* net, const char* path);

/* Forward pass over the batch's samples: y_dev (device [batch][4]) receives
 * the scaled outputs. */
int seb_net_forward(seb_net* net, const seb_train_batch* batch, float* y_dev, void* stream);

/* One training step on the batch: loss = mean over samples of the squared
 * error of the four scaled outputs against the labels (targets
 * ((z - h_ref)/0.05, roll/0.5, pitch/0.5, risk), where h_ref is the
 * sample cell's height when known, else the mean of its known in-map
 * 8-neighbours; every sample must have one); backward pass; Adam
 * (lr, beta 0.9 / 0.999, eps 1e-8) on float32 master weights.  loss_dev
 * (device float, may be NULL) receives the batch loss.  If grad_dev (device
 * [param_count]) is non-NULL the gradient is written there and the weights
 * are NOT updated. */
int seb_net_train_step(seb_net* net, const seb_train_batch* batch, float lr, float* loss_dev,
                       float* grad_dev, void* stream);
const char* seb_net_last_error(void);

/* Surrogate inference over a whole map with the plain method as fallback.
 * seb_surrogate_create allocates the workspace for ctx's map size (conv maps,
 * per-cell features, a one-byte fallback mark per state); release with
 * seb_surrogate_destroy.  The network must have been trained for ctx's
 * configuration (resolution, footprint, yaw bins, constants).  Errors:
 * SEB_ERR_INVALID, SEB_ERR_ALLOC, SEB_ERR_UNSUPPORTED (more than 128 yaw
 * units, i.e. n_yaw > 256 when even, > 128 when odd). */
typedef struct seb_surrogate seb_surrogate;
int seb_surrogate_create(seb_ctx* ctx, seb_surrogate** out);
void seb_surrogate_destroy(seb_surrogate* s);

/* Fill `out` ([K][H][W]) for every state of the map `height` ([H][W], row
 * stride ld).  Network outputs are written with status SEB_ST_VALID |
 * SEB_ST_SURROGATE (| SEB_ST_TRAV when risk <= risk_max).  A state falls back
 * to the plain method (Alg. 1 exactly as seb_assess_se2 computes it) when
 * neither its own cell nor any of its 8 neighbours is known (no reference
 * height for z: the own cell's, else the mean of the known neighbours), when
 * fewer than min_known of the 24 x 24 window's cells are known (outside the
 * training distribution), or when the predicted risk
 * lies within `band` of risk_max.  *n_fallback_dev (device int32, may be NULL)
 * receives the number of states that fell back.  Asynchronous on `stream`;
 * allocates nothing.  One surrogate handle serves one stream at a time. */
int seb_surrogate_infer(seb_surrogate* s, const seb_net* net, const float* height, int64_t ld,
                        const seb_out* out, float band, float min_known, int32_t* n_fallback_dev,
                        void* stream);

/* --------------------------------------------- elevation-map update */

/* One LiDAR scan and the frames and noise model of Sec. V-A, Eq. 5-9.
 * Matrices are row-major 3 x 3 rotations; positions in metres. */
typedef struct seb_scan {
    const float* points;     /* device [n_points][3] float32, sensor frame              */
    int64_t n_points;
    double R_B[9], p_B[3];   /* robot pose: body frame -> map frame                     */
    double R_BS[9], p_BS[3]; /* sensor extrinsics: sensor frame -> body frame           */
    double Sigma_R[9];       /* covariance of the body-frame rotation perturbation
                                R_B Exp(d) (rad^2), as in Eq. 7                          */
    double Sigma_B[9];       /* covariance of p_B (m^2); Eq. 9 uses its (2, 2) entry    */
    double sigma_range;      /* sensor model (> 0): range noise along the beam (m)      */
    double sigma_angle;      /* sensor model (>= 0): angular noise across it (rad)      */
    double z_min, z_max;     /* body-frame height band of the points kept               */
    double mahalanobis;      /* gate tau (> 0) of the several-heights rule              */
} seb_scan;

/* Workspace for fusing scans of up to max_points points into maps of ctx's
 * size (W * H < 2^31).  Errors: SEB_ERR_INVALID, SEB_ERR_UNSUPPORTED, SEB_ERR_ALLOC. */
typedef struct seb_fuser seb_fuser;
int seb_fuser_create(seb_ctx* ctx, int64_t max_points, seb_fuser** out);
void seb_fuser_destroy(seb_fuser* f);

/* Fuse one scan into the elevation map (Sec. V-A).  height and variance:
 * device [H][W] float32, row stride ld, in the ring storage of a window whose
 * logical cell (0, 0) is world cell (origin_x, origin_y) (world cell (gx, gy)
 * at position (gx mod W, gy mod H); origin (0, 0) is a plain map).  Each point
 * goes to the map frame (Sec. V-A: map rotation I, world cell = floor(x /
 * res)); it is dropped outside the window or outside the body-frame height
 * band; its height variance follows Eq. 5-9 with the sensor covariance
 * sigma_range^2 u u^T + (sigma_angle r)^2 (I - u u^T) (u the beam direction,
 * r the range).  The points of a cell then update it in increasing point
 * index with a one-dimensional Kalman filter, in FP64: an unknown cell
 * (non-finite height) takes the point; a point whose Mahalanobis distance
 * |z - h| / sqrt(v) exceeds tau replaces the cell if it is higher and is
 * dropped if it is lower (several heights in one cell); otherwise
 * h <- (v z + s h) / (v + s), v <- v s / (v + s).  Cells without points are
 * not touched; height and variance must not overlap.  *n_fused_dev (device
 * int32, may be NULL) receives the number of points that changed a cell.
 * Errors (host-side, nothing launched): SEB_ERR_INVALID.  Allocates nothing;
 * one fuser serves one stream at a time. */
int seb_fuse_scan(seb_fuser* f, float* height, float* variance, int64_t ld, int64_t origin_x,
                  int64_t origin_y, const seb_scan* scan, int32_t* n_fused_dev, void* stream);

/* seb_fuse_scan for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with the workspace in a file-scope device array of
 * about 10 MiB that every GPU the library runs on holds until the process
 * ends, instead of a seb_fuser.  Limits: W * H <= 2^18 cells and n_points <=
 * 2^18 (larger calls fail with SEB_ERR_INVALID, nothing launched).  The first
 * call on a device looks up the array's address there (SEB_ERR_HIP if that
 * fails).  All calls on one GPU share the array, so calls that overlap on one
 * GPU (several streams or threads) race; serialise them.  Arguments, ring
 * storage, n_fused_dev and errors as for seb_fuse_scan; allocates nothing. */
int seb_fuse_scan_static(seb_ctx* ctx, float* height, float* variance, int64_t ld,
                         int64_t origin_x, int64_t origin_y, const seb_scan* scan,
                         int32_t* n_fused_dev, void* stream);

/* Ray-casting reset (Sec. V-A), run before the scan is fused: every finite
 * point's segment from the sensor (R_B p_BS + p_B) to the point, in the map
 * frame, resets to unknown (NaN) each known cell it crosses -- a cell whose
 * interior its xy projection enters, i.e. whose slab-clipped parameter
 * interval satisfies t0 < t1 -- other than the point's own cell, when the
 * cell's height exceeds the segment's highest z over the crossing,
 * max(z(t0), z(t1)), by more than margin (metres, >= 0; 0 is the literal
 * test).  Decisions use the heights before the call, so the result does not
 * depend on ray order.  height: device [H][W] float32, row stride ld, ring
 * storage of the window whose logical (0, 0) is world cell (origin_x,
 * origin_y), as for seb_fuse_scan; only scan->points, n_points, R_B, p_B,
 * R_BS and p_BS are read.  *n_reset_dev (device int32, may be NULL) receives
 * the number of cells reset.  Errors: SEB_ERR_INVALID.  Allocates nothing. */
int seb_raycast_reset(seb_ctx* ctx, float* height, int64_t ld, int64_t origin_x, int64_t origin_y,
                      const seb_scan* scan, double margin, int32_t* n_reset_dev, void* stream);

/* Nearest-neighbour inpainting (the method the experiments use; Sec. V-A
 * leaves the inpainter open): every unknown (non-finite) cell of `height`
 * takes the height of the known cell with the smallest (dx^2 + dy^2, dy, dx)
 * within `radius` cells (0 <= radius <= 16), in logical coordinates; with none
 * it is written as NaN.  Known cells are copied.  height: device [H][W], row
 * stride ld; out: device [H][W], row stride out_ld, not overlapping height;
 * both in ring storage with offsets (ring_x, ring_y) as for seb_sdf_se2.
 * Errors: SEB_ERR_INVALID.  Allocates nothing. */
int seb_inpaint_nearest(seb_ctx* ctx, const float* height, int64_t ld, int32_t ring_x,
                        int32_t ring_y, int32_t radius, float* out, int64_t out_ld, void* stream);

/* ------------------------------------------- planner-side fields */

/* Signed distance field over the SE(2) states (Sec. V, and the safety
 * constraint of the trajectory optimisation, Sec. VI-B): for every state, the
 * distance in metres from its cell centre to the edge of the nearest obstacle
 * region within its own yaw plane, negative for states inside an obstacle.
 * Obstacle states are those with SEB_ST_CURV or SEB_ST_TILT set (Algorithm 1's
 * explicit obstacles), those with SEB_ST_SURROGATE set and SEB_ST_TRAV clear
 * (the surrogate does not tell which early-out applies, so every state it
 * answers as not traversable counts as an obstacle, the safe side), plus,
 * when unknown_is_obstacle != 0, UNKNOWN states (SEB_ST_VALID clear).  With d the Euclidean distance between cell centres
 * (in cells) to the nearest obstacle state (for a free state) or nearest free
 * state (for an obstacle state), and C = cap_cells,
 *     sdf = +(min(d, C) - 0.5) res   (free),   -(min(d, C) - 0.5) res   (obstacle);
 * a plane with no obstacle (or no free) state gives the capped value.  Cells
 * outside the map are neither.
 * status / sdf: device [K][H][W] of ctx's map, both in ring storage: logical
 * cell (x, y) at position ((x + ring_x) mod W, (y + ring_y) mod H), so the
 * arrays of a rolling window can be passed as they are (ring_x = ring_y = 0
 * for a plain map).  Errors (host-side, nothing launched): SEB_ERR_INVALID
 * (NULL array, ring offset outside [0, W) x [0, H), cap_cells < 1),
 * SEB_ERR_UNSUPPORTED (cap_cells > 64, or W * H >= 2^31).  Enqueues one
 * kernel; allocates nothing. */
int seb_sdf_se2(seb_ctx* ctx, const uint8_t* status, int32_t ring_x, int32_t ring_y,
                int32_t cap_cells, int32_t unknown_is_obstacle, float* sdf, void* stream);

/* Trilinear interpolation of the SDF and of the risk at arbitrary poses, with
 * the yaw axis on SO(2) (Sec. VI-B/VI-C: the planner reads both fields and
 * their gradients along the trajectory).  poses: device [n][3] float32
 * (x, y, theta) in logical map metres, the corner of cell (0, 0) at the
 * origin (cell (i, j)'s centre at ((i + 0.5) res, (j + 0.5) res)), yaw bin k
 * at theta = 2 pi k / K.  out: device [n][8] float32 = (sdf, dsdf/dx,
 * dsdf/dy, dsdf/dtheta, risk, drisk/dx, drisk/dy, drisk/dtheta).  A position
 * outside the cell centres' range is clamped onto it (the derivative along a
 * clamped axis is 0); theta wraps; derivatives are those of the trilinear
 * cell [floor, floor + 1] that holds the pose.  NaN coordinates read as the
 * clamped lower edge and yaw bin 0.  sdf and risk: device [K][H][W] in the
 * ring storage of seb_sdf_se2; either may be NULL (its four outputs are then
 * 0), not both.  out must be 16-byte aligned.  n == 0 is a no-op.  Errors:
 * SEB_ERR_INVALID.  Allocates nothing. */
int seb_query_se2(seb_ctx* ctx, const float* sdf, const float* risk, int32_t ring_x, int32_t ring_y,
                  const float* poses, int64_t n, float* out, void* stream);

/* --------------------------------------------------------------- misc */

const char* seb_strerror(int status);
const char* seb_last_error(void);
const char* seb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SEB_H */
