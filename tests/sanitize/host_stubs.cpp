// Host stand-ins for building libseb's host code without the GPU, for the
// address / undefined-behaviour sanitizer test: the kernel launchers report
// that there is no device, and the five HIP runtime calls the host code makes
// work on host memory.  Test infrastructure only.
#include <cstdlib>
#include <cstring>

#include <hip/hip_runtime.h>

#include "seb_elevation_internal.hpp"
#include "seb_internal.hpp"
#include "seb_net_internal.hpp"
#include "seb_sdf_internal.hpp"
#include "seb_surrogate_internal.hpp"

extern "C" {
hipError_t hipMalloc(void** p, size_t bytes) {
    *p = std::malloc(bytes ? bytes : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "host stand-in"; }
}

namespace seb {
hipError_t launch_assess(const AssessArgs&, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_assess_flagged(const AssessArgs&, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_insert(const InsertArgs&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_sdf(const uint8_t*, float*, int, int, int, int, int, int, float, int, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_query(const float*, const float*, const float*, float*, int64_t, int, int, int,
                        int, int, double, hipStream_t) {
    return hipErrorNoDevice;
}
namespace net {
const float* net_theta(const seb_net*) { return nullptr; }
PackedWeights net_packed(const seb_net*) { return PackedWeights{}; }
}  // namespace net
namespace sur {
hipError_t launch_surrogate(const SurArgs&, const AssessArgs&, hipStream_t) { return hipErrorNoDevice; }
}  // namespace sur
namespace elev {
hipError_t launch_fuse_scan(const ScanArgs&, const FuseArgs&, const FuseWork&, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_raycast(const RayArgs&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_inpaint(const InpaintArgs&, hipStream_t) { return hipErrorNoDevice; }
hipError_t static_fuse_work(FuseWork*) { return hipErrorNoDevice; }
}  // namespace elev
}  // namespace seb
