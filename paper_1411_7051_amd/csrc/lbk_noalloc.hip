// lbk_noalloc.hip -- the global permeability read-out for callers that cannot
// allocate: lbk_apparent_permeability_noalloc computes what
// lbk_apparent_permeability does, but keeps its FP64 partial sums and
// results in a fixed device array of this file instead of the lattice's
// workspace and its pinned host buffer, and calls no allocating routine.
//
// The array `scratch` below holds one partial per read-out slot for each of
// at most kGrid workgroups, then the slots' totals.  Each GPU the library
// runs on holds its own copy until the process ends.  In host code the
// array's name is only a stand-in for the symbol: its device address, one
// per device, comes from hipGetSymbolAddress on the first call on that
// device (with the device current) and is what every launch and copy uses.
//
// Every partial and total is written before it is read in each call, so
// nothing needs clearing between calls; but all calls on one GPU share the
// array, so calls that overlap in time on one GPU (several host threads, or
// lattices on different streams) race and must be serialized by the caller.
#include "lbk_host.h"

#include <mutex>

namespace lbk {
namespace {

// Workgroups of the strided read-out: enough to fill the 256 compute units
// several times over, few enough that the partials stay small.
constexpr int kGrid = 2048;
constexpr size_t kScratchDoubles = (size_t)(kGrid + 1) * MAC_SLOTS;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices]; // device address of `scratch`, per device

// Device address of this device's `scratch` (dev must be current).
lbk_status scratch_of(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LBK_ERR_UNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBK_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s",
                        hipGetErrorString(e));
        g_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_ptr[dev];
    return LBK_OK;
}

// Makes `dev` current for the lifetime of the object and restores the
// device that was current before.
struct DeviceGuard {
    int prev = -1;
    bool switched = false;
    hipError_t enter(int dev)
    {
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess || prev == dev)
            return e;
        e = hipSetDevice(dev);
        switched = e == hipSuccess;
        return e;
    }
    ~DeviceGuard()
    {
        if (switched)
            (void)hipSetDevice(prev);
    }
};

} // namespace
} // namespace lbk

using namespace lbk;

extern "C" lbk_status lbk_apparent_permeability_noalloc(lbk_lattice *lat, double *k_app)
{
    if (!lat || !k_app)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    if (!has_drive(lat->d))
        return fail(LBK_ERR_INVALID_ARG, "the global permeability needs rho_in != rho_out "
                                         "(pressure drive) or gx != 0");
    const Launch l = launch_of(lat->g);
    const int grid = l.blocks < kGrid ? l.blocks : kGrid;
    // partials [MAC_SLOTS][grid], then the MAC_SLOTS totals
    const size_t need = (size_t)(grid + 1) * MAC_SLOTS;
    if (grid < 1 || need > kScratchDoubles)
        return fail(LBK_ERR_UNSUPPORTED, "read-out needs %zu doubles of scratch, %zu available",
                    need, kScratchDoubles);
    DeviceGuard guard;
    HIP_TRY(guard.enter(lat->device));
    double *base = nullptr;
    lbk_status s = scratch_of(lat->device, &base);
    if (s != LBK_OK)
        return s;
    double *partials = base;
    double *totals = base + (size_t)grid * MAC_SLOTS;
    const lbk_desc &d = lat->d;
    HIP_TRY(launch_macro_strided(d.storage, d.bc_x, d.bc_y, lat->state(lat->cur), lat->L.lay,
                                 lat->med(), lat->L.mlay, lat->g, lat->ph, lat->s(),
                                 lat->inv_s(), grid, partials, lat->stream));
    HIP_TRY(launch_finish(partials, MAC_SLOTS, grid, 0, totals, lat->stream));
    double sums[MAC_SLOTS];
    HIP_TRY(hipMemcpyAsync(sums, totals, sizeof sums, hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    *k_app = k_app_of(lat, sums);
    return LBK_OK;
}
