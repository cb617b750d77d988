// Elevation-map update before the assessment (seb_elevation.hip): point
// variance and cell assignment, per-cell Kalman fusion, nearest-neighbour
// inpainting.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace seb {
namespace elev {

constexpr int INPAINT_MAX_RADIUS = 16;
constexpr int INPAINT_MAX_OFFS = 832;     // >= offsets with 0 < dx^2 + dy^2 <= 16^2 (796)

// One scan: points, frames and noise model, written as the per-point
// arithmetic needs them (J_S and g = R_B^T b3 precomputed on the host).
struct ScanArgs {
    const float* pts;        // [n][3] sensor frame
    int64_t n;
    double A[9], a[3];       // R_BS (row-major), p_BS
    double R[9], b[3];       // R_B, p_B
    double js[3];            // J_S = (R_B R_BS)^T b3
    double g[3];             // R_B^T b3
    double SR[9];            // Sigma_R
    double sb22;             // Sigma_B[2][2]
    double sr2, sa2;         // sigma_range^2, sigma_angle^2
    double zmin, zmax, res;
    int32_t W, H;
    int64_t ox, oy;          // world cell of logical (0, 0)
};

// Workspace of one fuser (sized at creation).
struct FuseWork {
    int32_t* cell;           // [max_points] logical cell or -1
    double* z;               // [max_points]
    double* var;             // [max_points]
    int32_t* bucket;         // [max_points] point indices grouped by cell
    int32_t* count;          // [W*H]
    int32_t* fill;           // [W*H]
    int32_t* offs;           // [W*H] exclusive prefix sum of count
    int32_t* partial;        // [partial_blocks(W*H)]
    int32_t* large;          // [W*H] cells with more points than a thread folds alone
    int32_t* n_large;        // [1]
    int32_t* n_fused;        // [1] internal counter when the caller passes none
};

constexpr int SCAN_CHUNK = 4096;          // cells per prefix-sum block (256 x 16)
inline int64_t partial_blocks(int64_t n_cells) { return (n_cells + SCAN_CHUNK - 1) / SCAN_CHUNK; }

// Limits of seb_fuse_scan_static, whose workspace is a file-scope device array.
constexpr int64_t STATIC_MAX_POINTS = int64_t(1) << 18;
constexpr int64_t STATIC_MAX_CELLS = int64_t(1) << 18;
// The FuseWork buffers inside that array on the current device (its address
// is looked up once per device, on the first call there).  Allocates nothing.
hipError_t static_fuse_work(FuseWork* w);

struct FuseArgs {
    float* height;           // [H][ld] ring storage
    float* variance;
    int64_t ld;
    int32_t W, H, rx, ry;    // ring offsets = origin mod size
    double tau2;             // Mahalanobis threshold squared
    int32_t* n_fused;        // device counter (points that changed a cell)
};

hipError_t launch_fuse_scan(const ScanArgs& s, const FuseArgs& f, const FuseWork& w,
                            hipStream_t stream);

// Ray-casting reset: the scan's rays against the heights in ring storage.
struct RayArgs {
    const float* pts;        // [n][3] sensor frame
    int64_t n;
    double A[9], a[3];       // R_BS, p_BS
    double R[9], b[3];       // R_B, p_B
    double sx, sy, sz;       // sensor origin R_B p_BS + p_B (map frame)
    double res, margin;
    int32_t W, H, rx, ry;
    int64_t ox, oy;          // world cell of logical (0, 0)
    float* height;           // [H][ld] ring storage
    int64_t ld;
    int32_t* n_reset;        // device counter or null
};

hipError_t launch_raycast(const RayArgs& r, hipStream_t stream);

struct InpaintArgs {
    const float* src;        // [H][ld] ring storage
    int64_t ld;
    float* dst;              // [H][dst_ld] ring storage, same offsets
    int64_t dst_ld;
    int32_t W, H, rx, ry;
    int32_t radius;
    const int2* offs;        // (dx, dy) sorted by (dx^2 + dy^2, dy, dx)
    int32_t n_offs;          // entries with dx^2 + dy^2 <= radius^2
};

hipError_t launch_inpaint(const InpaintArgs& a, hipStream_t stream);

}  // namespace elev
}  // namespace seb
