// fm_apply_operator_noalloc: the operator of fm_apply_operator with its scratch
// (the energies on the device and the two coupling slots) in a static device
// array instead of library allocations, for callers that cannot allocate.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "fm_problem.h"

namespace {

constexpr size_t SCRATCH_DOUBLES = size_t(8) << 20;   // 64 MiB per GPU
constexpr size_t E_SLOTS = 4096;                        // energies: the first 32 KiB

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on device dev, which must be current; looked up
// on the first call on that device and kept.
hipError_t scratch_on(int dev, double **out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

fm_status nfail(fm_status s, const std::string &m) {
    fm::set_error(m);
    return s;
}

}  // namespace

extern "C" fm_status fm_apply_operator_noalloc(fm_problem *p, int nbatch, const double *E, const double *x_dev,
                                               double *y_dev, void *stream) {
    if (!p || !E || !x_dev || !y_dev || nbatch < 1) return nfail(FM_E_INVALID, "bad argument");
    if (x_dev == y_dev) return nfail(FM_E_INVALID, "x and y must not overlap");
    if (size_t(nbatch) > E_SLOTS)
        return nfail(FM_E_INVALID, "nbatch exceeds the allocation-free limit of 4096 requests");
    const size_t slots = 2 * size_t(nbatch) * size_t(p->N);
    if (slots > SCRATCH_DOUBLES - E_SLOTS)
        return nfail(FM_E_INVALID, "2 * nbatch * N = " + std::to_string(slots) +
                                       " doubles exceed the allocation-free scratch of " +
                                       std::to_string(SCRATCH_DOUBLES - E_SLOTS) + " doubles");
    const int dev = p->desc.device;
    if (dev < 0 || dev >= MAX_DEVICES) return nfail(FM_E_INVALID, "device ordinal out of range");
    fm::Busy busy(p);
    if (!busy.ok) return nfail(FM_E_BUSY, "problem handle in use");
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return nfail(FM_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    double *base = nullptr;
    e = scratch_on(dev, &base);
    if (e != hipSuccess) return nfail(FM_E_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *E_dev = base;
    double *cbuf = base + E_SLOTS;
    e = hipMemcpyAsync(E_dev, E, sizeof(double) * nbatch, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return nfail(FM_E_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    // the coupling writes only the slots of points that have coupling pairs;
    // the others must read zero, whatever an earlier call left in the array
    fm::launch_fill(cbuf, (long long)slots, 0.0, st);
    fm::launch_matvec(p->pd, nbatch, E_dev, nullptr, x_dev, y_dev, cbuf, st, 2);
    fm::launch_matvec(p->pd, nbatch, E_dev, nullptr, x_dev, y_dev, cbuf, st, 1);
    e = hipGetLastError();
    if (e != hipSuccess) return nfail(FM_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return nfail(FM_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    return FM_OK;
}
