// HIP kernels for gfx950: SE(2)-grid traversability assessment (Sec. V-B,
// Algorithm 1, with the pose of Sec. III, Eq. 1-3) and rolling-window cell
// insertion (Sec. V-A).
//
// Work decomposition.  A workgroup stages the heights of a 16 x 16 block of
// states plus an R-cell halo into LDS once, then loops over yaw bins; each
// lane owns one state (cell) and walks the footprint samples of the current
// yaw bin in table order.  The table entry of a sample (LDS offset, bilinear
// weights, body coordinates) is the same for every lane, so the whole wave
// reads it with scalar loads and the FMAs take it as a scalar operand.  Lanes
// map to 16 consecutive x-cells of 4 rows, which with a row pitch of 16 mod 32
// floats keeps every LDS read conflict-free.
//
// Yaw bins k and k + K/2 sample exactly the same map points with body
// coordinates negated, so one pass yields both: height, curvature, tilt and
// risk are shared, roll and pitch change sign.
//
// Per-state arithmetic.  Heights are centred on a per-state reference (the
// state's own cell, else the first valid sample in table order) before the
// moments are summed in FP32.  The exact integer moments of the valid sample
// positions (N, sum p, sum q, sum p^2, sum pq, sum q^2) give an exact gate
// (enough samples, not collinear) and exact centred second moments; the
// least-squares plane is then a closed-form 2 x 2 solve.
#include <cmath>

#include "seb.h"
#include "seb_internal.hpp"
#include "seb_state_device.hpp"

namespace seb {
namespace {

using namespace dev;

// The least-squares kernels are held to 8 waves per SIMD (64 VGPRs), which
// the chunked sample loop would otherwise exceed by one register; the FP64
// eigen epilogue of the principal-component fit needs more and runs at 5.
template <int P, int NW, int FIT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(FIT == 0 ? 8 : 1)))
void assess_kernel(const AssessArgs a) {
    extern __shared__ float tile[];
    const int tid = threadIdx.x;

    // Which rectangle and which tile of it.
    const int b = blockIdx.x;
    int ri = 0;
    while (ri + 1 < a.n_rects && b >= a.tile_start[ri + 1]) ++ri;
    const int lb = b - a.tile_start[ri];
    const int tyi = lb / a.tiles_x[ri];
    const int txi = lb - tyi * a.tiles_x[ri];
    const int sx0 = a.rect[ri][0] + txi * TILE;
    const int sy0 = a.rect[ri][1] + tyi * TILE;
    const int sx1 = a.rect[ri][0] + a.rect[ri][2];
    const int sy1 = a.rect[ri][1] + a.rect[ri][3];
    const int R = a.R;
    const int tw = TILE + 2 * R;

    // Stage heights of logical cells [sx0-R, sx0+16+R) x [sy0-R, sy0+16+R).
    for (int i = tid; i < tw * tw; i += BLOCK) {
        const int ly = i / tw;
        const int lx = i - ly * tw;
        const int gx = sx0 - R + lx, gy = sy0 - R + ly;
        float v = SENTINEL;
        if (gx >= 0 && gx < a.W && gy >= 0 && gy < a.H) {
            const int px = wrap(gx + a.rx, a.W), py = wrap(gy + a.ry, a.H);
            const float h = a.height[(int64_t)py * a.ld + px];
            if (fabsf(h) < HEIGHT_LIMIT) v = h;      // false for NaN and +-Inf
        }
        tile[ly * P + lx] = v;
    }
    __syncthreads();

    const int lane = tid & 63;
    const int lx = lane & 15;
    const int ly = (tid >> 6) * 4 + (lane >> 4);
    const int ix = sx0 + lx, iy = sy0 + ly;
    const bool active = ix < sx1 && iy < sy1;
    const float* tp0 = tile + (ly + R) * P + (lx + R);
    const float hc = tp0[0];
    const int64_t cell = (int64_t)wrap(iy + a.ry, a.H) * a.W + wrap(ix + a.rx, a.W);

    const int u0 = blockIdx.y * a.units_per_group;
    const int u1 = min(a.n_units, u0 + a.units_per_group);
    for (int u = u0; u < u1; ++u) {
        const Result r = assess_state<NW, FIT>(a, LdsSource<P>{tp0}, u, hc, active);
        if (active) {
            store(a, u, cell, r, false);
            if (a.mirror) store(a, u + a.mirror, cell, r, true);
        }
    }
}

// Re-assessment of the states flagged in a.need only.  The map is cut into
// TF x TF blocks; a block's flagged cells of one yaw unit form a list in cell
// order, and workgroup (block, slice, unit) assesses list entries
// [256 slice, 256 slice + 256): it builds the list (ballot and prefix sum,
// so every slice sees the same order), returns before staging when its slice
// is empty, stages the block's heights once and lets each lane assess one
// listed state.  No lane is spent on an unflagged state, no wave assesses more
// than one state, and the footprint table stays wave-uniform.  The per-state
// arithmetic is assess_kernel's, so results are identical.
template <int P, int NW, int FIT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(FIT == 0 ? 8 : 1)))
void assess_flagged_kernel(const AssessArgs a, const int TF) {
    extern __shared__ float tile[];
    __shared__ int wave_n[BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int R = a.R;
    const int tw = TF + 2 * R;
    uint16_t* list = (uint16_t*)(tile + tw * P);
    const int slices = TF * TF / BLOCK;
    const int blk = blockIdx.x / slices, slice = blockIdx.x - blk * slices;
    const int tiles_x = (a.W + TF - 1) / TF;
    const int sx0 = (blk % tiles_x) * TF, sy0 = (blk / tiles_x) * TF;
    const int u = blockIdx.y;
    const int64_t plane = (int64_t)a.W * a.H;

    // Flagged cells of the block in cell order.
    int n = 0;
    for (int i0 = 0; i0 < TF * TF; i0 += BLOCK) {
        const int i = i0 + tid;
        const int ly = i / TF, lx = i - ly * TF;
        const int ix = sx0 + lx, iy = sy0 + ly;
        bool f = false;
        if (ix < a.W && iy < a.H) {
            const int64_t c = (int64_t)wrap(iy + a.ry, a.H) * a.W + wrap(ix + a.rx, a.W);
            f = a.need[(int64_t)u * plane + c] != 0;
        }
        const uint64_t m = __ballot(f);
        if (lane == 0) wave_n[wave] = __popcll(m);
        __syncthreads();
        int before = n;
        for (int w = 0; w < wave; ++w) before += wave_n[w];
        if (f) list[before + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)i;
        for (int w = 0; w < BLOCK / 64; ++w) n += wave_n[w];
        __syncthreads();
    }
    if (slice == 0 && tid == 0 && a.count && n > 0) atomicAdd(a.count, n * (a.mirror ? 2 : 1));
    const int first = slice * BLOCK;
    if (n <= first) return;

    for (int i = tid; i < tw * tw; i += BLOCK) {
        const int ly = i / tw;
        const int lx = i - ly * tw;
        const int gx = sx0 - R + lx, gy = sy0 - R + ly;
        float v = SENTINEL;
        if (gx >= 0 && gx < a.W && gy >= 0 && gy < a.H) {
            const int px = wrap(gx + a.rx, a.W), py = wrap(gy + a.ry, a.H);
            const float h = a.height[(int64_t)py * a.ld + px];
            if (fabsf(h) < HEIGHT_LIMIT) v = h;
        }
        tile[ly * P + lx] = v;
    }
    __syncthreads();

    const int i = first + tid;
    const bool act = i < n;
    if (!__ballot(act)) return;
    const int li = list[act ? i : first];
    const int ly = li / TF, lx = li - ly * TF;
    const int ix = sx0 + lx, iy = sy0 + ly;
    const float* tp0 = tile + (ly + R) * P + (lx + R);
    const int64_t cell = (int64_t)wrap(iy + a.ry, a.H) * a.W + wrap(ix + a.rx, a.W);
    const Result r = assess_state<NW, FIT>(a, LdsSource<P>{tp0}, u, tp0[0], act);
    if (act) {
        store(a, u, cell, r, false);
        if (a.mirror) store(a, u + a.mirror, cell, r, true);
    }
}

// Write newly exposed cells (or unknown) into the ring.
__global__ __launch_bounds__(BLOCK) void insert_kernel(const InsertArgs a) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int lx, ly;
    float v;
    if (a.full) {
        if (i >= (int64_t)a.W * a.H) return;
        ly = (int)(i / a.W);
        lx = (int)(i - (int64_t)ly * a.W);
        v = a.src ? a.src[(int64_t)ly * a.src_ld + lx] : __builtin_nanf("");
    } else {
        const int64_t nrow = (int64_t)a.rows_n * a.W;
        const int rem = a.H - a.rows_n;
        if (i < nrow) {
            ly = a.rows_lo + (int)(i / a.W);
            lx = (int)(i % a.W);
        } else {
            const int64_t j = i - nrow;
            if (a.cols_n == 0 || j >= (int64_t)a.cols_n * rem) return;
            const int r = (int)(j / a.cols_n);
            ly = (a.rows_lo == 0 ? a.rows_n : 0) + r;
            lx = a.cols_lo + (int)(j - (int64_t)r * a.cols_n);
        }
        v = a.src ? a.src[i] : __builtin_nanf("");
    }
    const int px = wrap(lx + a.rx, a.W), py = wrap(ly + a.ry, a.H);
    a.ring[(int64_t)py * a.ld + px] = v;
}

}  // namespace

int pick_pitch(int R) {
    const int need = TILE + 2 * R;
    static const int pitches[] = {48, 80, 112, 144};
    for (int p : pitches)
        if (p >= need) return p;
    return 0;
}

bool has_row_kernel(int row_len) { return row_len == 4 || row_len == 12 || row_len == 24; }

template <int P, int FIT>
static void launch_pf(const AssessArgs& a, dim3 grid, size_t lds, hipStream_t stream) {
    switch (a.row_len) {
        case 4: hipLaunchKernelGGL((assess_kernel<P, 4, FIT>), grid, dim3(BLOCK), lds, stream, a); break;
        case 12: hipLaunchKernelGGL((assess_kernel<P, 12, FIT>), grid, dim3(BLOCK), lds, stream, a); break;
        case 24: hipLaunchKernelGGL((assess_kernel<P, 24, FIT>), grid, dim3(BLOCK), lds, stream, a); break;
        default: hipLaunchKernelGGL((assess_kernel<P, 0, FIT>), grid, dim3(BLOCK), lds, stream, a); break;
    }
}

template <int P>
static hipError_t launch_p(const AssessArgs& a, dim3 grid, size_t lds, hipStream_t stream) {
    if (a.fit == 1)
        launch_pf<P, 1>(a, grid, lds, stream);
    else
        launch_pf<P, 0>(a, grid, lds, stream);
    return hipGetLastError();
}

hipError_t launch_assess(const AssessArgs& a, int pitch, hipStream_t stream) {
    const int tiles = a.tile_start[a.n_rects];
    if (tiles == 0) return hipSuccess;
    const int groups = (a.n_units + a.units_per_group - 1) / a.units_per_group;
    const dim3 grid(tiles, groups);
    const size_t lds = (size_t)(TILE + 2 * a.R) * pitch * sizeof(float);
    switch (pitch) {
        case 48: return launch_p<48>(a, grid, lds, stream);
        case 80: return launch_p<80>(a, grid, lds, stream);
        case 112: return launch_p<112>(a, grid, lds, stream);
        case 144: return launch_p<144>(a, grid, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

template <int P, int FIT>
static void launch_flagged_pf(const AssessArgs& a, int tf, dim3 grid, size_t lds, hipStream_t stream) {
    switch (a.row_len) {
        case 4: hipLaunchKernelGGL((assess_flagged_kernel<P, 4, FIT>), grid, dim3(BLOCK), lds, stream, a, tf); break;
        case 12: hipLaunchKernelGGL((assess_flagged_kernel<P, 12, FIT>), grid, dim3(BLOCK), lds, stream, a, tf); break;
        case 24: hipLaunchKernelGGL((assess_flagged_kernel<P, 24, FIT>), grid, dim3(BLOCK), lds, stream, a, tf); break;
        default: hipLaunchKernelGGL((assess_flagged_kernel<P, 0, FIT>), grid, dim3(BLOCK), lds, stream, a, tf); break;
    }
}

template <int P>
static hipError_t launch_flagged_p(const AssessArgs& a, int tf, dim3 grid, size_t lds,
                                   hipStream_t stream) {
    if (a.fit == 1)
        launch_flagged_pf<P, 1>(a, tf, grid, lds, stream);
    else
        launch_flagged_pf<P, 0>(a, tf, grid, lds, stream);
    return hipGetLastError();
}

int flagged_tile(int R, int pitch) { return (32 + 2 * R <= pitch) ? 32 : 16; }

hipError_t launch_assess_flagged(const AssessArgs& a, int pitch, hipStream_t stream) {
    if (!a.need || a.W <= 0 || a.H <= 0 || a.n_units <= 0) return hipErrorInvalidValue;
    const int tf = flagged_tile(a.R, pitch);
    const int tiles = ((a.W + tf - 1) / tf) * ((a.H + tf - 1) / tf);
    const dim3 grid(tiles * (tf * tf / BLOCK), a.n_units);
    const size_t lds = (size_t)(tf + 2 * a.R) * pitch * sizeof(float) + (size_t)tf * tf * 2;
    switch (pitch) {
        case 48: return launch_flagged_p<48>(a, tf, grid, lds, stream);
        case 80: return launch_flagged_p<80>(a, tf, grid, lds, stream);
        case 112: return launch_flagged_p<112>(a, tf, grid, lds, stream);
        case 144: return launch_flagged_p<144>(a, tf, grid, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_insert(const InsertArgs& a, hipStream_t stream) {
    int64_t n = a.full ? (int64_t)a.W * a.H
                       : (int64_t)a.rows_n * a.W + (int64_t)a.cols_n * (a.H - a.rows_n);
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(insert_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

}  // namespace seb
