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

// The footprint table, structure of arrays, sample order = rows of constant
// body-x index i, each row in increasing body-y index j:
//   wts  [n_units][n_samples] float4  bilinear weights of corners (0,0) (1,0) (0,1) (1,1)
//   offs [n_units][n_samples] int32   LDS offset dy * pitch + dx of corner (0,0)
//   frac [n_units][n_samples] double2 FP64 fractions (fx, fy) for the FP64 path
//   qs   [n_samples] float, pks [n_samples] uint32: body-y index q = 2j - (nw-1)
//        and the packed (1, q + qoff, q^2) of the exact integer moments
// All entries of one sample are the same for every lane of a wave, which
// reads them with scalar loads.

// A run of samples sharing the body-x index p (one row of the sample grid, or
// a piece of it short enough for the packed integer moments not to overflow).
struct Segment {
    int32_t p;        // body-x sample index p = 2i - (nl-1)
    int32_t count;
    int32_t first;    // index of the first sample of the run within a yaw bin
    int32_t pad;
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
    // footprint table (see above)
    const float4* wts;
    const int32_t* offs;
    const double2* frac;
    const float* qs;
    const uint32_t* pks;
    const Segment* segs;         // [n_segs]
    int32_t row_len;             // samples per segment when every segment is a full
                                 // row of the rectangle (fast path), else 0
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
    float inv_hu, inv_hv;        // 1 / hu, 1 / hv
    double rho16;                // near-degenerate threshold (rho of full footprint / 16)
    int32_t n_total;             // samples in the full footprint
    float kappa_max, phi_x_max, phi_y_max, w_kappa, w_phi_x, w_phi_y, risk_max;
    float c_kappa, c_phi_x, c_phi_y;   // w_kappa / kappa_max, w_phi_x / phi_x_max, w_phi_y / phi_y_max
    int32_t min_valid;
    int32_t precision;
    int32_t fit;                 // 0 least-squares plane, 1 principal-component plane
    int32_t* count;              // optional, zero on entry: the flagged-state
                                 // kernel adds the number of states it assesses
                                 // (both mirror bins)
    // Flagged states, listed row by row per (unit, block) of TF x TF cells
    // (TF = flagged_tile), slot = unit * blocks + block: row r of the slot's
    // block lists row_count[slot * TF + r] block-local columns at
    // work_cols[(slot * TF + r) * TF ..].  Rows past the map's edge count zero.
    const uint8_t* row_count;
    const uint8_t* work_cols;
    // state rectangles (logical coordinates) and their tile decomposition
    int32_t n_rects;
    int32_t rect[MAX_RECTS][4];
    int32_t tiles_x[MAX_RECTS];
    int32_t tiles_y[MAX_RECTS];
    // A rect whose last tile column holds at most 8 columns runs that column as
    // pairs of vertically adjacent tiles, one workgroup per pair (lanes 0-7 the
    // upper tile, lanes 8-15 the lower), after its full tiles.
    int32_t edge_pair[MAX_RECTS];
    int32_t tile_start[MAX_RECTS + 1];
    // Ring insert of a window move, fused into the assessment (ins_on, never
    // with ins.full): the exposed cells are staged from ins.src instead of the
    // ring, and ins_blocks x gridDim.y more workgroups, after the tiles, write
    // them into the ring.  The ring cells they overwrite lie outside the new
    // window, so no workgroup of the launch reads them.
    InsertArgs ins;
    int32_t ins_on, ins_blocks;
};

// Launchers (seb_assess.hip).  Return hipSuccess or the launch error.
hipError_t launch_assess(const AssessArgs& a, int pitch, hipStream_t stream);
// Assess only the states listed in a.row_count / a.work_cols, anywhere in the
// map, 64 listed states per workgroup.
hipError_t launch_assess_flagged(const AssessArgs& a, int pitch, hipStream_t stream);
// Block side of the flagged-state kernels: 32 when its halo fits the pitch.
inline int flagged_tile(int R, int pitch) { return (32 + 2 * R <= pitch) ? 32 : 16; }
inline int64_t flagged_blocks(int W, int H, int n_units, int R, int pitch) {   // units x blocks
    const int tf = flagged_tile(R, pitch);
    return (int64_t)((W + tf - 1) / tf) * ((H + tf - 1) / tf) * n_units;
}
inline int64_t flagged_work_items(int W, int H, int n_units, int R, int pitch) {
    const int tf = flagged_tile(R, pitch);
    return flagged_blocks(W, H, n_units, R, pitch) * (tf * tf / 64);
}
// Row lengths with a specialised (fully unrolled) inner loop.
inline bool has_row_kernel(int row_len) { return row_len == 4 || row_len == 12 || row_len == 24; }
hipError_t launch_insert(const InsertArgs& a, hipStream_t stream);
// LDS pitches (floats) the assessment kernel is instantiated for: the
// smallest that holds a tile plus its halo, 0 if none does.
inline int pick_pitch(int R) {
    const int need = TILE + 2 * R;
    for (int p : {48, 80, 112, 144})
        if (p >= need) return p;
    return 0;
}
// LDS bytes of a workgroup that runs a pair of edge tiles.
inline size_t edge_pair_lds(int R, int pitch) {
    return (size_t)2 * (TILE + 2 * R) * pitch * sizeof(float);
}

}  // namespace seb
