// Allocation-free variant of lbib_get_macros for callers that cannot allocate device memory
// (tight serving loops, harnesses that forbid hipMalloc).  lbib_get_macros stages the moments
// in a device buffer it allocates per call; this variant stages them in a fixed array of device
// memory that the library holds from load time on every GPU it runs on.
#include "lbib.h"
#include "lbib_runtime.h"

#include <mutex>

namespace {

// 4 doubles per node (rho, u*_x, u*_y, u*_z), LBIB_NOALLOC_MAX_NODES nodes: 32 MiB per GPU.
// In host code this name is only a stand-in for the symbol; the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[4 * (size_t)LBIB_NOALLOC_MAX_NODES];

constexpr int kMaxDevices = 64;
std::mutex g_dev_lock[kMaxDevices];          // serialises the calls on one device
double* g_scratch_ptr[kMaxDevices] = {};     // device address of scratch, per device

// Device address of this device's copy of scratch (the device must be current).  Looked up on
// the first call on the device and kept; the caller holds g_dev_lock[dev].
lbib_status scratch_on(int dev, double** out) {
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return lbib::fail_static(LBIB_EDEVICE, "hipGetSymbolAddress of the scratch array failed");
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return LBIB_OK;
}

lbib_status get_macros_locked(lbib::Batch& B, int job, int dev, double* rho, double* u) {
    using lbib::fail_static;
    double* ptr = nullptr;
    lbib_status st = scratch_on(dev, &ptr);
    if (st) return st;
    // deferred errors of the queued steps, as lbib_get_macros reports them: the flags of every
    // job of the batch, read through a fixed host buffer
    if (hipStreamSynchronize(B.stream) != hipSuccess) return fail_static(LBIB_EDEVICE, "stream synchronisation failed");
    const int njobs = (int)B.jobs.size();
    int fl[256];
    for (int j0 = 0; j0 < njobs; j0 += 256) {
        const int cnt = njobs - j0 < 256 ? njobs - j0 : 256;
        if (hipMemcpy(fl, B.P.flags + j0, sizeof(int) * cnt, hipMemcpyDeviceToHost) != hipSuccess)
            return fail_static(LBIB_EDEVICE, "reading the job flags failed");
        for (int j = 0; j < cnt; ++j) {
            if (fl[j] & lbib::FLAG_NONFINITE) return fail_static(LBIB_EUNSTABLE, "a job of this batch has a non-finite or runaway state");
            if (fl[j] & lbib::FLAG_DOMAIN) return fail_static(LBIB_EDOMAIN, "a job of this batch has an MLS support or probe on a wall");
            if (fl[j] & lbib::FLAG_WINDOW) return fail_static(LBIB_EDOMAIN, "a body of this batch outgrew its window");
        }
    }
    const long long n = B.jobs[job].n;
    // every entry of the 4n doubles is written, so nothing of the previous call is read
    lbib::launch_macros_f64(B.P, B.storage, B.cur_b, job, n, ptr, B.stream);
    if (hipGetLastError() != hipSuccess) return fail_static(LBIB_EDEVICE, "macro kernel launch failed");
    if (rho && hipMemcpyAsync(rho, ptr, sizeof(double) * n, hipMemcpyDeviceToHost, B.stream) != hipSuccess)
        return fail_static(LBIB_EDEVICE, "copy of rho failed");
    if (u && hipMemcpyAsync(u, ptr + n, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, B.stream) != hipSuccess)
        return fail_static(LBIB_EDEVICE, "copy of u failed");
    if (hipStreamSynchronize(B.stream) != hipSuccess) return fail_static(LBIB_EDEVICE, "stream synchronisation failed");
    return LBIB_OK;
}

}  // namespace

extern "C" lbib_status lbib_get_macros_noalloc(lbib_lattice* lat, double* rho, double* u) {
    using lbib::fail_static;
    if (!lat || !lat->batch) return fail_static(LBIB_EINVAL, "null lattice handle");
    lbib::Batch& B = *lat->batch;
    if (B.jobs[lat->job].n > LBIB_NOALLOC_MAX_NODES)
        return fail_static(LBIB_EINVAL, "lattice larger than LBIB_NOALLOC_MAX_NODES (1048576 nodes); use lbib_get_macros");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail_static(LBIB_EDEVICE, "hipGetDevice failed");
    if (dev != B.device) return fail_static(LBIB_EINVAL, "the lattice's device must be the current device");
    if (dev < 0 || dev >= kMaxDevices) return fail_static(LBIB_EINVAL, "device index beyond the library's table");
    try {
        std::lock_guard<std::mutex> hold(g_dev_lock[dev]);
        return get_macros_locked(B, lat->job, dev, rho, u);
    } catch (...) {
        return fail_static(LBIB_EDEVICE, "device lock failed");
    }
}
