// pbs_bind_static: bind a context to a scratch array that the library holds in device memory, for
// callers that cannot allocate device memory themselves (see include/pbsplit.h).
//
// The array is a file-scope __device__ variable, so every GPU the library runs on holds its own copy
// (PBS_STATIC_SCRATCH_BYTES, until the process ends).  Host code never passes the array's name to a
// kernel or a copy: its device address is looked up once per device with hipGetSymbolAddress and kept
// here, and only that address is used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "pbs_common.h"
#include "pbs_ctx.h"
#include "pbsplit.h"

static __device__ __align__(256) unsigned char scratch[PBS_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};                    // device address of `scratch` per device (null: not looked up)
unsigned long long g_epoch[MAX_DEVICES] = {};     // number of static binds per device

}  // namespace

bool pbs::static_lost(const pbs_ctx *c)
{
    if (c->static_dev < 0 || c->static_dev >= MAX_DEVICES) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_epoch[c->static_dev] != c->static_epoch;
}

extern "C" pbs_status pbs_bind_static(pbs_ctx *c, void *hip_stream)
{
    if (!c) return PBS_EINVAL;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return pbs::ctx_fail(c, PBS_EDEVICE, (std::string("hipGetDevice: ") + hipGetErrorString(e)).c_str());
    if (dev < 0 || dev >= MAX_DEVICES) return pbs::ctx_fail(c, PBS_EUNSUPPORTED, "device index beyond 63");
    if (c->total > (size_t)PBS_STATIC_SCRATCH_BYTES) {
        const std::string m = "workspace of " + std::to_string(c->total) + " bytes exceeds the static scratch of " +
                              std::to_string((size_t)PBS_STATIC_SCRATCH_BYTES) + " bytes";
        return pbs::ctx_fail(c, PBS_EINVAL, m.c_str());
    }
    void *ptr = nullptr;
    unsigned long long epoch = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_ptr[dev]) {
            // the current device is `dev`: its copy of the array
            e = hipGetSymbolAddress(&g_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess || !g_ptr[dev]) {
                g_ptr[dev] = nullptr;
                return pbs::ctx_fail(c, PBS_EDEVICE,
                                     (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
            }
        }
        ptr = g_ptr[dev];
        epoch = ++g_epoch[dev];
    }
    c->static_dev = dev;
    c->static_epoch = epoch;
    // every buffer that must start at zero is cleared by pbs_set_beam (fluence, source scans, dose); the
    // tables are written here
    return pbs::bind_workspace(c, static_cast<char *>(ptr), (size_t)PBS_STATIC_SCRATCH_BYTES,
                               (hipStream_t)hip_stream, false);
}
