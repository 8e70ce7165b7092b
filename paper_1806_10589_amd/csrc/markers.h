// roctx ranges on the host side of the library's launches, switched on by
// FLBM_PROFILE=1 at context creation. The roctx library is opened at run
// time (rocprofiler-sdk's, which rocprofv3 --marker-trace records, else the
// older libroctx64), so the library has no link dependency on it; when
// neither is found the ranges are no-ops.
#pragma once
#include <dlfcn.h>

#include <mutex>

namespace flbm {

struct Roctx {
    typedef int (*push_fn)(const char *);
    typedef int (*pop_fn)();
    push_fn push = nullptr;
    pop_fn pop = nullptr;

    static const Roctx &get()
    {
        static Roctx r;
        static std::once_flag once;
        std::call_once(once, [] {
            const char *names[] = {"librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so",
                                   "libroctx64.so.4", "libroctx64.so"};
            for (const char *n : names) {
                void *h = dlopen(n, RTLD_NOW | RTLD_LOCAL);
                if (!h) continue;
                r.push = (push_fn)dlsym(h, "roctxRangePushA");
                r.pop = (pop_fn)dlsym(h, "roctxRangePop");
                if (r.push && r.pop) break;
                r.push = nullptr;
                r.pop = nullptr;
            }
        });
        return r;
    }
};

// A named range for the lifetime of the object, when `on`.
class Range {
public:
    Range(bool on, const char *name) : on_(on && Roctx::get().push)
    {
        if (on_) Roctx::get().push(name);
    }
    ~Range()
    {
        if (on_) Roctx::get().pop();
    }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;

private:
    bool on_;
};

}  // namespace flbm
