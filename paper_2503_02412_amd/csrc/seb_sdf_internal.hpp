// Launchers of the signed distance field and the trilinear query (seb_sdf.hip).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace seb {

// Ring offsets (rx, ry) map logical cell (x, y) to storage position
// ((x + rx) mod W, (y + ry) mod H); 0 <= rx < W and 0 <= ry < H.
inline int sdf_max_cap() { return 64; }   // largest cap (cells) the kernel's LDS halo is sized for
hipError_t launch_sdf(const uint8_t* status, float* sdf, int W, int H, int K, int rx, int ry,
                      int cap, float res, int unknown_is_obstacle, hipStream_t stream);
hipError_t launch_query(const float* fa, const float* fb, const float* poses, float* out, int64_t n,
                        int W, int H, int K, int rx, int ry, double res, hipStream_t stream);

}  // namespace seb
