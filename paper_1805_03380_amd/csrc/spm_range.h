// Optional roctx ranges around the entry points that launch work (host code).  With the
// environment variable SPM_ROCTX set to a non-empty value other than "0", every such call is
// pushed as a range named after the entry point, so a rocprofv3 run with --marker-trace shows
// which call each kernel belongs to.  roctx is looked up with dlopen on the first call: the
// library does not depend on it, and without the variable (or without a roctx library) a
// range costs one branch.
#pragma once

#include <dlfcn.h>

#include <cstdlib>
#include <initializer_list>

namespace spm {

struct RoctxFns {
  int (*push)(const char*);
  int (*pop)();
};

inline const RoctxFns& roctx_fns() {
  static const RoctxFns fns = [] {
    RoctxFns r{nullptr, nullptr};
    const char* e = std::getenv("SPM_ROCTX");
    if (!e || !*e || (e[0] == '0' && e[1] == '\0')) return r;
    // the profiler SDK's roctx first (rocprofv3 --marker-trace records its ranges), then the
    // older library of the same interface
    void* h = nullptr;
    for (const char* lib : {"librocprofiler-sdk-roctx.so", "librocprofiler-sdk-roctx.so.1",
                            "libroctx64.so", "libroctx64.so.4"}) {
      h = dlopen(lib, RTLD_NOW | RTLD_LOCAL);
      if (h) break;
    }
    if (!h) return r;
    r.push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    r.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!r.push || !r.pop) r = RoctxFns{nullptr, nullptr};
    return r;
  }();
  return fns;
}

// One range for the lifetime of the object (the whole entry point, every return path).
class Range {
 public:
  explicit Range(const char* name) : on_(roctx_fns().push != nullptr) {
    if (on_) roctx_fns().push(name);
  }
  ~Range() {
    if (on_) roctx_fns().pop();
  }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;

 private:
  bool on_;
};

}  // namespace spm

#define SPM_RANGE(name) ::spm::Range spm_range_guard_(name)
