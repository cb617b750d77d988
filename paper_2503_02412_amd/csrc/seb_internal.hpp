// Internal declarations shared by the host code and the HIP kernels of the
// SE(2) traversability library.  Not part of the public C ABI (include/seb.h).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace seb {

// One workgroup assesses a TILE x TILE block of states: four wave64s, each
// covering 16 consecutive x-cells of 4 consecutive rows.
constexpr int TILE = 16;
constexpr int BLOCK = 256;
constexpr int MAX_RECTS = 8;

// LDS stand-in for an unknown or out-of-map cell.  Any bilinear sample that
// gives it a nonzero weight (>= 1e-12 once fractions near integers are
// snapped) lands above VALID_LIMIT, while a zero weight cancels it exactly;
// so |sample - ref| < VALID_LIMIT is the validity rule "every corner with
// nonzero weight is known".  Known heights must satisfy |h| < HEIGHT_LIMIT.
constexpr float SENTINEL = 0x1p110f;
constexpr float VALID_LIMIT = 0x1p64f;
constexpr float HEIGHT_LIMIT = 0x1p60f;

// One footprint sample of one yaw bin.  32 bytes; read by the whole wave at
// once through the scalar unit.
struct TblEntry {
    int32_t off;                 // LDS offset (dy * pitch + dx) of the lower-left corner
    float w00, w01, w10, w11;    // bilinear weights of corners (0,0) (1,0) (0,1) (1,1)
    float q;                     // body-y sample index q = 2j - (nw-1), as float
    uint32_t pk;                 // packed (1, q + qoff, q^2) for exact integer moments
    int32_t pad;
};

// A run of samples sharing the body-x index p (one row of the sample grid, or
// a piece of it short enough for the packed integer moments not to overflow).
struct Segment {
    int32_t p;        // body-x sample index p = 2i - (nl-1)
    int32_t count;
    int32_t first;    // index of the first sample of the run within a yaw bin
    int32_t pad;
};

struct AssessArgs {
    // map (ring storage) and outputs
    const float* height;
    int64_t ld;
    int32_t W, H;
    int32_t rx, ry;              // ring offset: logical (x, y) lives at ((x+rx)%W, (y+ry)%H)
    float* z;
    float* roll;
    float* pitch;
    float* risk;
    uint8_t* status;
    // footprint table
    const TblEntry* tbl;         // [n_units][n_samples]
    const double2* frac;         // [n_units][n_samples] FP64 (fx, fy) for the FP64 path
    const Segment* segs;         // [n_segs]
    int32_t n_units;             // yaw bins computed directly
    int32_t mirror;              // K/2 when yaw bin k+K/2 is derived from bin k, else 0
    int32_t n_samples;
    int32_t n_segs;
    int32_t K;
    int32_t R;                   // halo (cells) of the LDS tile
    int32_t units_per_group;
    // packed integer moments of a segment: bits [0,6) count, [6, 6+w1) sum of
    // (q + qoff), [sh2, 32) sum of q^2.
    int32_t qoff;
    uint32_t mask1;
    int32_t sh2;
    float hu, hv;                // metres per unit of p and of q
    double rho16;                // near-degenerate threshold (rho of full footprint / 16)
    int32_t n_total;             // samples in the full footprint
    float kappa_max, phi_x_max, phi_y_max, w_kappa, w_phi_x, w_phi_y, risk_max;
    int32_t min_valid;
    int32_t precision;
    // state rectangles (logical coordinates) and their tile decomposition
    int32_t n_rects;
    int32_t rect[MAX_RECTS][4];
    int32_t tiles_x[MAX_RECTS];
    int32_t tile_start[MAX_RECTS + 1];
};

struct InsertArgs {
    float* ring;
    int64_t ld;
    int32_t W, H;
    int32_t rx, ry;              // ring offset of the NEW window
    const float* src;            // exposed cells in plan order, or null (unknown)
    int64_t src_ld;              // for full copies: row stride of src
    int32_t rows_lo, rows_n;     // exposed row strip [rows_lo, rows_lo + rows_n)
    int32_t cols_lo, cols_n;     // exposed column strip
    int32_t full;                // 1: copy the whole logical window from src
};

// Launchers (seb_assess.hip).  Return hipSuccess or the launch error.
hipError_t launch_assess(const AssessArgs& a, int pitch, hipStream_t stream);
hipError_t launch_insert(const InsertArgs& a, hipStream_t stream);
// LDS pitches (floats) the assessment kernel is instantiated for.
int pick_pitch(int R);

}  // namespace seb
