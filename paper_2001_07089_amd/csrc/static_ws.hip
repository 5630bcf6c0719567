// static_ws.hip -- a context whose workspace is a fixed device array, for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The array `scratch` below exists once per GPU the library runs on and is
// held until the process ends.  In host code its name only stands for the
// device object: its device address is taken with hipGetSymbolAddress, once
// per device with that device current, and only that address is handed on.
// md_init zeroes every part of a workspace that its kernels read before they
// write it, so what an earlier context left in the array does not matter.
// One context at a time may use a device's array: a second md_init_static on
// that device is refused until the first context is destroyed (two contexts
// in one array would overwrite each other's state).
#include <cstdio>
#include <mutex>

#include "kamd_internal.hpp"

namespace {

constexpr size_t STATIC_WS_BYTES = (size_t)64 << 20;  // 64 MiB: ~43,000 particles with 16 MSD slots
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) char scratch[STATIC_WS_BYTES];

std::mutex g_mutex;
void *g_addr[MAX_DEVICES];   // device address of `scratch` on each device, once taken
bool g_in_use[MAX_DEVICES];  // a live context works in that device's array

}  // namespace

namespace kamd {
void release_static_workspace(int device)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (device >= 0 && device < MAX_DEVICES) g_in_use[device] = false;
}
}  // namespace kamd

extern "C" int md_init_static(kamd_ctx **out, const kamd_config *cfg, const kamd_replica *reps, int32_t n_rep,
                              const kamd_state *st, void *hip_stream)
{
    char msg[256];
    if (!out) {
        kamd::set_init_error("out is null");
        return KAMD_EINVAL;
    }
    *out = nullptr;
    size_t need = 0;
    int rc = md_workspace_size(cfg, reps, n_rep, &need);
    if (rc) return rc;
    if (need > STATIC_WS_BYTES) {
        snprintf(msg, sizeof msg, "md_init_static: this configuration needs %zu bytes of workspace, "
                                  "more than the %zu of the static array (use md_init)", need, STATIC_WS_BYTES);
        kamd::set_init_error(msg);
        return KAMD_ENOMEM;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        kamd::set_init_error("md_init_static: no usable current HIP device");
        return KAMD_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_in_use[dev]) {
        snprintf(msg, sizeof msg, "md_init_static: a context already works in the static array of device %d "
                                  "(md_destroy it first)", dev);
        kamd::set_init_error(msg);
        return KAMD_ESTATE;
    }
    if (!g_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            snprintf(msg, sizeof msg, "md_init_static: hipGetSymbolAddress: %s", hipGetErrorString(e));
            kamd::set_init_error(msg);
            return KAMD_EHIP;
        }
        g_addr[dev] = p;
    }
    rc = md_init(out, cfg, reps, n_rep, st, g_addr[dev], STATIC_WS_BYTES, hip_stream);
    if (rc == KAMD_OK) {
        g_in_use[dev] = true;
        kamd::mark_static(*out, dev);
    }
    return rc;
}
