// Optional roctx ranges for profiler timelines (rocprofv3 --marker-trace). With
// NKREG_ROCTX=1 in the environment the library opens ROCm's roctx library at run time
// and names its calls, solver iterations and (eager) transport sweeps; otherwise, or
// when the library is missing, a range costs one branch. Ranges are host-side: inside a
// replayed graph they mark when the host enqueued it.
#pragma once

#include <dlfcn.h>

#include <cstdlib>
#include <string>

namespace nk {

struct Roctx {
  using PushFn = int (*)(const char*);
  using PopFn = int (*)();
  PushFn push = nullptr;
  PopFn pop = nullptr;
  static const Roctx& get() {
    static const Roctx r = load();
    return r;
  }

 private:
  static Roctx load() {
    Roctx r;
    const char* e = std::getenv("NKREG_ROCTX");
    if (!e || e[0] != '1') return r;
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("librocprofiler-sdk-roctx.so", RTLD_NOW | RTLD_LOCAL);
    if (!h) return r;
    r.push = reinterpret_cast<PushFn>(dlsym(h, "roctxRangePushA"));
    r.pop = reinterpret_cast<PopFn>(dlsym(h, "roctxRangePop"));
    if (!r.push || !r.pop) r.push = nullptr, r.pop = nullptr;
    return r;
  }
};

// A roctx range for the lifetime of the object.
class Range {
 public:
  explicit Range(const char* name) : on_(Roctx::get().push != nullptr) {
    if (on_) Roctx::get().push(name);
  }
  Range(const char* name, int k) : on_(Roctx::get().push != nullptr) {
    if (on_) Roctx::get().push((std::string(name) + " " + std::to_string(k)).c_str());
  }
  ~Range() {
    if (on_) Roctx::get().pop();
  }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;

 private:
  bool on_;
};

}  // namespace nk
