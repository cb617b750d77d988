// roctx ranges around the C-ABI calls, so that a profile (rocprofv3
// --marker-trace) shows each call of the library as a named range around its
// kernels.  The roctx library is opened on first use; without it every range
// is a no-op, and with it but no profiler attached a range costs two calls
// into it.
#pragma once

#include <dlfcn.h>

#include <cstdlib>
#include <string>

namespace seb {

struct TraceApi {
    int (*push)(const char*) = nullptr;
    int (*pop)() = nullptr;
};

inline const TraceApi& trace_api() {
    static const TraceApi api = [] {
        TraceApi t;
        const char* root = std::getenv("ROCM_PATH");
        const std::string dir = std::string(root && *root ? root : "/opt/rocm") + "/lib/";
        const std::string names[] = {"librocprofiler-sdk-roctx.so.1", dir + "librocprofiler-sdk-roctx.so.1"};
        for (const std::string& n : names) {
            void* h = dlopen(n.c_str(), RTLD_NOW | RTLD_LOCAL);
            if (!h) continue;
            t.push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
            t.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
            if (t.push && t.pop) break;
            t.push = nullptr;
            t.pop = nullptr;
        }
        return t;
    }();
    return api;
}

class TraceRange {
  public:
    explicit TraceRange(const char* name) : on_(trace_api().push != nullptr) {
        if (on_) trace_api().push(name);
    }
    ~TraceRange() {
        if (on_) trace_api().pop();
    }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;

  private:
    bool on_;
};

}  // namespace seb

// A range named after the enclosing C-ABI function, for the rest of its body.
#define SEB_TRACE_RANGE() ::seb::TraceRange seb_trace_range_(__func__)
