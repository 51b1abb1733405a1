// Named host ranges for ROCm's tracing tools (roctx).  Each C ABI call that
// enqueues device work opens a range for the duration of its enqueue, so a
// marker trace (rocprofv3 --marker-trace) shows which call launched which
// kernels.  The roctx library is opened at the first range; where it is
// missing, or SW_ROCTX=0 is set, ranges do nothing.
#include <dlfcn.h>

#include <cstdlib>
#include <mutex>

#include "runtime.h"

namespace sw {

namespace {

using PushFn = int (*)(const char *);
using PopFn = int (*)();
PushFn g_push = nullptr;
PopFn g_pop = nullptr;
std::once_flag g_once;

void open_roctx()
{
    const char *env = std::getenv("SW_ROCTX");
    if (env && env[0] == '0') return;
    void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    auto push = reinterpret_cast<PushFn>(dlsym(h, "roctxRangePushA"));
    auto pop = reinterpret_cast<PopFn>(dlsym(h, "roctxRangePop"));
    if (push && pop) {
        g_push = push;
        g_pop = pop;
    }
}

}  // namespace

Range::Range(const char *name)
{
    std::call_once(g_once, open_roctx);
    if (g_push) {
        g_push(name);
        active_ = true;
    }
}

Range::~Range()
{
    if (active_) g_pop();
}

}  // namespace sw
