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
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "seb.h"
#include "seb_internal.hpp"
#include "seb_state_device.hpp"

namespace seb {
namespace {

using namespace dev;

// The least-squares kernels are held to 8 waves per SIMD (64 VGPRs), which
// the chunked sample loop would otherwise exceed by one register; the FP64
// eigen epilogue of the principal-component fit needs more and runs at 5.
// Cell i of a move's exposed cells (in plan order: the exposed row strip row
// by row, then the exposed column strip), or of the whole window for a full
// copy, written into the ring.
__device__ __forceinline__ void insert_cell(const InsertArgs& a, int64_t i) {
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

// Height of logical cell (gx, gy) of a window being moved: an exposed cell's
// from the move's source (NaN without one), any other from the ring.
__device__ __forceinline__ float moved_height(const AssessArgs& a, int gx, int gy) {
    const InsertArgs& s = a.ins;
    int64_t i = -1;
    if (gy >= s.rows_lo && gy < s.rows_lo + s.rows_n)
        i = (int64_t)(gy - s.rows_lo) * s.W + gx;
    else if (gx >= s.cols_lo && gx < s.cols_lo + s.cols_n)
        i = (int64_t)s.rows_n * s.W + (int64_t)(gy - (s.rows_lo == 0 ? s.rows_n : 0)) * s.cols_n +
            (gx - s.cols_lo);
    if (i >= 0) return s.src ? s.src[i] : __builtin_nanf("");
    return a.height[(int64_t)wrap(gy + a.ry, a.H) * a.ld + wrap(gx + a.rx, a.W)];
}

template <int P, int NW, int FIT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(FIT == 0 ? 8 : 1)))
void assess_kernel(const AssessArgs a) {
    extern __shared__ float tile[];
    const int tid = threadIdx.x;

    // Which rectangle and which tile of it.
    const int b = blockIdx.x;
    if (b >= a.tile_start[a.n_rects]) {           // the fused ring insert
        insert_cell(a.ins, ((int64_t)(b - a.tile_start[a.n_rects]) * gridDim.y + blockIdx.y) * BLOCK + tid);
        return;
    }
    int ri = 0;
    while (ri + 1 < a.n_rects && b >= a.tile_start[ri + 1]) ++ri;
    const int lb = b - a.tile_start[ri];
    const int tx = a.tiles_x[ri];
    int txi, tyi;
    bool paired = false;
    if (a.edge_pair[ri] && lb >= (tx - 1) * a.tiles_y[ri]) {
        paired = true;                             // tiles tyi and tyi + 1 of the last column
        txi = tx - 1;
        tyi = 2 * (lb - (tx - 1) * a.tiles_y[ri]);
    } else {
        const int w = a.edge_pair[ri] ? tx - 1 : tx;
        tyi = lb / w;
        txi = lb - tyi * w;
    }
    const int sx0 = a.rect[ri][0] + txi * TILE;
    const int sy0 = a.rect[ri][1] + tyi * TILE;
    const int sx1 = a.rect[ri][0] + a.rect[ri][2];
    const int sy1 = a.rect[ri][1] + a.rect[ri][3];
    const int R = a.R;
    const int tw = TILE + 2 * R;

    // Stage heights of logical cells [sx0-R, sx0+16+R) x [sy0-R, sy0+16+R); a
    // pair stages [sx0-R, sx0+8+R) of both tiles, the lower one tw rows further
    // down and 8 columns further right in LDS (so that lanes 8-15 fall on the
    // banks next to lanes 0-7).
    const int cw = paired ? TILE / 2 + 2 * R : tw;
    const int n_stage = (paired ? 2 : 1) * tw * cw;
    auto stage = [&](auto moved) {
        for (int i = tid; i < n_stage; i += BLOCK) {
            const int half = i >= tw * cw;
            const int k = i - half * tw * cw;
            const int ly = k / cw;
            const int lx = k - ly * cw;
            const int gx = sx0 - R + lx, gy = sy0 - R + ly + half * TILE;
            float v = SENTINEL;
            if (gx >= 0 && gx < a.W && gy >= 0 && gy < a.H) {
                float h;
                if constexpr (decltype(moved)::value) {
                    h = moved_height(a, gx, gy);
                } else {
                    const int px = wrap(gx + a.rx, a.W), py = wrap(gy + a.ry, a.H);
                    h = a.height[(int64_t)py * a.ld + px];
                }
                if (fabsf(h) < HEIGHT_LIMIT) v = h;      // false for NaN and +-Inf
            }
            tile[(half * tw + ly) * P + lx + half * (TILE / 2)] = v;
        }
    };
    if (a.ins_on)
        stage(std::true_type{});
    else
        stage(std::false_type{});
    __syncthreads();

    const int lane = tid & 63;
    const int lx = lane & 15;
    const int ly = (tid >> 6) * 4 + (lane >> 4);
    const int hb = paired ? lx >> 3 : 0;           // lower tile of a pair
    const int ix = sx0 + (paired ? lx & 7 : lx), iy = sy0 + ly + hb * TILE;
    const bool active = ix < sx1 && iy < sy1;
    if (!__ballot(active)) return;                 // wave entirely past the rectangle's edge
    const float* tp0 = tile + (hb * tw + ly + R) * P + (lx + R);
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

// Re-assessment of the listed (flagged) states only.
//
// flagged_kernel: one workgroup per possible item of 64 listed states,
// item-major (workgroup k * slots + slot takes item k of slot (unit, block)),
// so the first items of every block come first and workgroups past a block's
// count return at once.  A slot's states are its rows' lists in row order;
// the workgroup finds its 64 from the slot's row counts (a prefix sum over the
// lanes and a binary search), takes their bounding box (wave reductions) and
// stages the box plus the footprint halo.  Its first workgroups also add the
// listed states to the optional state counter, 2048 words of four row counts
// per workgroup and one atomic add per wave.  Each of its four waves
// accumulates a quarter of the footprint rows for the same 64 states; wave 0
// adds the four partial moment sets and finishes the states.  Four short
// waves per 64 states keep many more SIMDs busy than one long wave would, for
// the few thousand states a map sends back.  A state whose own cell is
// unknown takes, in each wave, the first valid sample of that wave's rows as
// reference; the partial sums are shifted exactly onto the first wave's
// reference (the first valid sample in table order):
//   S(z - r) = S(z - r_w) + N_w d,  S q(z - r) = S q(z - r_w) + d S q,
//   S (z - r)^2 = S (z - r_w)^2 + 2 d S(z - r_w) + N_w d^2,  d = r_w - r.
template <int P, int NW, int FIT>
__global__ __launch_bounds__(BLOCK) void flagged_kernel(const AssessArgs a, const int TF) {
    extern __shared__ float tile[];
    // Partial moments of waves 1..3: in FP32 mode the tile is dead once the
    // moments are summed, so they reuse its start (after a barrier); the FP64
    // redo reads the tile later, so with precision 1 they sit after it.
    const size_t tile_words = (size_t)(TF + 2 * a.R) * P;
    Parts& parts = *reinterpret_cast<Parts*>(a.precision == 1 ? tile + tile_words : tile);
    // The wave index, and with it the wave's footprint rows and every table
    // address, marked wave-uniform so the table arrives by scalar loads.
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int R = a.R;
    const int tiles_x = (a.W + TF - 1) / TF;
    const int nr = a.n_segs;
    const int g0 = nr * wave / 4, g1 = nr * (wave + 1) / 4;
    {
        const int blocks = tiles_x * ((a.H + TF - 1) / TF);
        const int nslot = blocks * a.n_units;
        const int nwords = nslot * TF / 4;       // row counts, four per word
        if (a.count && (int64_t)blockIdx.x * (BLOCK * 8) < nwords) {
            // Workgroup b sums words [2048 b, 2048 b + 2048): eight loads per
            // thread in flight, then one add per wave to the counter.
            const uint32_t* words = reinterpret_cast<const uint32_t*>(a.row_count);
            int total = 0;
            const int q0 = blockIdx.x * (BLOCK * 8) + tid;
            uint32_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = words[min(q0 + BLOCK * j, nwords - 1)];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                total += q0 + BLOCK * j < nwords ? (int)((v[j] & 0xffu) + ((v[j] >> 8) & 0xffu) +
                                                         ((v[j] >> 16) & 0xffu) + (v[j] >> 24))
                                                  : 0;
            for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o);
            if (lane == 0 && total > 0) atomicAdd(a.count, total * (a.mirror ? 2 : 1));
        }
        const int k = blockIdx.x / nslot, slot = blockIdx.x % nslot;
        // Row counts of the slot on lanes 0..TF-1, inclusive prefix sums.
        const int rc = lane < TF ? (int)a.row_count[slot * TF + lane] : 0;
        int incl = rc;
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        const int cnt = __builtin_amdgcn_readfirstlane(__shfl(incl, TF - 1));
        if (64 * k >= cnt) return;
        const int u = slot / blocks, blk = slot % blocks;
        // List position of the lane's state (lanes past the count take the
        // item's first state: staged, not stored), its row (the first whose
        // inclusive prefix exceeds it) and its column.
        const bool act = 64 * k + lane < cnt;
        const int lp = act ? 64 * k + lane : 64 * k;
        int row = 0;
        for (int st = TF >> 1; st > 0; st >>= 1)
            if (__shfl(incl, row + st - 1) <= lp) row += st;
        const int start = __shfl(incl, row) - __shfl(rc, row);
        const int col = a.work_cols[((int64_t)slot * TF + row) * TF + (lp - start)];
        // Bounding box of the item's cells (wave reductions).
        int bx0 = col, by0 = row, bx1 = col, by1 = row;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            bx0 = min(bx0, __shfl_xor(bx0, o));
            by0 = min(by0, __shfl_xor(by0, o));
            bx1 = max(bx1, __shfl_xor(bx1, o));
            by1 = max(by1, __shfl_xor(by1, o));
        }
        bx0 = __builtin_amdgcn_readfirstlane(bx0);
        by0 = __builtin_amdgcn_readfirstlane(by0);
        bx1 = __builtin_amdgcn_readfirstlane(bx1);
        by1 = __builtin_amdgcn_readfirstlane(by1);
        const int bw = bx1 - bx0 + 1 + 2 * R;
        const int bh = by1 - by0 + 1 + 2 * R;
        const int li = row * TF + col;
        // Block origin moved to the bounding box of the item's cells.
        const int sx0 = (blk % tiles_x) * TF + bx0, sy0 = (blk / tiles_x) * TF + by0;
        // Staging: SB elements of the box per thread and batch, loaded from
        // clamped positions without a guard so the batch's loads are all in
        // flight together; out-of-map and unknown cells become SENTINEL.
        // A workgroup holds a few dozen states, so the latency of these loads,
        // not their bandwidth, is what the staging costs.
        constexpr int SB = 8;
        const int n = bw * bh;
        const float inv_bw = 1.f / (float)bw;
        for (int i0 = tid; i0 < n; i0 += BLOCK * SB) {
            float v[SB];
            int pos[SB];
            uint32_t ok = 0u;
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const int i = min(i0 + BLOCK * j, n - 1);
                // i / bw from the float quotient (i < 2^24), corrected by one either way
                int ly = (int)((float)i * inv_bw);
                ly += (i - ly * bw >= bw) ? 1 : 0;
                ly -= (i - ly * bw < 0) ? 1 : 0;
                const int lx = i - ly * bw;
                const int gy = sy0 - R + ly, gx = sx0 - R + lx;
                ok |= (uint32_t)(gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) << j;
                const int cy = min(max(gy, 0), a.H - 1), cx = min(max(gx, 0), a.W - 1);
                v[j] = a.height[(int64_t)wrap(cy + a.ry, a.H) * a.ld + wrap(cx + a.rx, a.W)];
                pos[j] = ly * P + lx;
            }
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const bool keep = ((ok >> j) & 1u) && fabsf(v[j]) < HEIGHT_LIMIT;  // false for NaN, Inf
                if (i0 + BLOCK * j < n) tile[pos[j]] = keep ? v[j] : SENTINEL;
            }
        }
        __syncthreads();
        const int ly = li / TF - by0, lx = li % TF - bx0;   // relative to the bounding box
        const float* tp0 = tile + (ly + R) * P + (lx + R);
        const float hc = tp0[0];
        float ref = (fabsf(hc) < HEIGHT_LIMIT) ? hc : 0.f;
        bool need = act && !(fabsf(hc) < HEIGHT_LIMIT);
        Moments<float> m;
        // Scattered lanes make every tile read a bank-conflicted one here, so
        // samples that repeat their predecessor's corner cell skip the reads.
        partial_moments<NW, LdsSource<P>, true>(a, LdsSource<P>{tp0}, u, g0, g1, ref, need, m);
        if (a.precision != 1) __syncthreads();    // every wave is done with the tile
        if (wave > 0) put_part(parts, wave, lane, m, ref, need);
        __syncthreads();
        if (wave == 0) {
            merge_parts(parts, 1, 3, lane, m, ref, need);
            const Result r = finish_state<FIT>(a, LdsSource<P>{tp0}, u, m, ref);
            if (act) {
                const int ix = sx0 + lx, iy = sy0 + ly;
                const int64_t cell = (int64_t)wrap(iy + a.ry, a.H) * a.W + wrap(ix + a.rx, a.W);
                store(a, u, cell, r, false);
                if (a.mirror) store(a, u + a.mirror, cell, r, true);
            }
        }
    }
}

// Write newly exposed cells (or unknown) into the ring.
__global__ __launch_bounds__(BLOCK) void insert_kernel(const InsertArgs a) {
    insert_cell(a, (int64_t)blockIdx.x * BLOCK + threadIdx.x);
}

}  // namespace

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
    const dim3 grid(tiles + (a.ins_on ? a.ins_blocks : 0), groups);
    bool any_pair = false;
    for (int r = 0; r < a.n_rects; ++r) any_pair = any_pair || a.edge_pair[r];
    const size_t lds = any_pair ? edge_pair_lds(a.R, pitch)
                                : (size_t)(TILE + 2 * a.R) * pitch * sizeof(float);
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
        case 4: hipLaunchKernelGGL((flagged_kernel<P, 4, FIT>), grid, dim3(BLOCK), lds, stream, a, tf); break;
        case 12: hipLaunchKernelGGL((flagged_kernel<P, 12, FIT>), grid, dim3(BLOCK), lds, stream, a, tf); break;
        case 24: hipLaunchKernelGGL((flagged_kernel<P, 24, FIT>), grid, dim3(BLOCK), lds, stream, a, tf); break;
        default: hipLaunchKernelGGL((flagged_kernel<P, 0, FIT>), grid, dim3(BLOCK), lds, stream, a, tf); break;
    }
}

template <int P>
static void launch_flagged_p(const AssessArgs& a, int tf, dim3 grid, size_t lds, hipStream_t stream) {
    if (a.fit == 1)
        launch_flagged_pf<P, 1>(a, tf, grid, lds, stream);
    else
        launch_flagged_pf<P, 0>(a, tf, grid, lds, stream);
}

hipError_t launch_assess_flagged(const AssessArgs& a, int pitch, hipStream_t stream) {
    if (!a.row_count || !a.work_cols || a.W <= 0 || a.H <= 0 || a.n_units <= 0) return hipErrorInvalidValue;
    if (pitch != 48 && pitch != 80 && pitch != 112 && pitch != 144) return hipErrorInvalidValue;
    const int tf = flagged_tile(a.R, pitch);
    // One workgroup per possible item; those past their block's count return.
    const int64_t max_items = flagged_work_items(a.W, a.H, a.n_units, a.R, pitch);
    const dim3 grid((unsigned)max_items);
    const size_t tile_bytes = (size_t)(tf + 2 * a.R) * pitch * sizeof(float);
    const size_t lds = a.precision == 1 ? tile_bytes + sizeof(Parts) : std::max(tile_bytes, sizeof(Parts));
    switch (pitch) {
        case 48: launch_flagged_p<48>(a, tf, grid, lds, stream); break;
        case 80: launch_flagged_p<80>(a, tf, grid, lds, stream); break;
        case 112: launch_flagged_p<112>(a, tf, grid, lds, stream); break;
        default: launch_flagged_p<144>(a, tf, grid, lds, stream); break;
    }
    return hipGetLastError();
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
