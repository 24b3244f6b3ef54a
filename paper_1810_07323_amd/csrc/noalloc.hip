// cor_utv_ex_noalloc: the single decomposition of cor_utv_ex run entirely in
// a fixed device array of this library, for callers that cannot allocate
// device memory.
//
// The array `scratch` below is a file-scope device variable: every device the
// library runs on holds its own copy (loaded with the code object, kept until
// the process ends).  Its name in host code is only a host-side stand-in, so
// host code never hands it to a kernel or a copy; the device address of each
// device's copy is looked up once per device with hipGetSymbolAddress (with
// that device current) and kept in `g_scratch`.  A call lays the plan (problem
// descriptor, launch tables, workspace) out in that memory, uploads the
// descriptor and tables, clears the workspace with a fill kernel, runs the
// same kernels as cor_utv_ex and waits for them.  It calls no hipMalloc,
// hipFree or other allocating device routine.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/cor_utv.h"
#include "common.h"
#include "runtime.h"

namespace cor {

// Fixed device memory of the no-allocation entry point (per device).
static __device__ __align__(256) unsigned char scratch[COR_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu[MAX_DEVICES];  // one call at a time per device
static void* g_scratch[MAX_DEVICES];          // device address of `scratch` per device
static std::once_flag g_scratch_once[MAX_DEVICES];
static hipError_t g_scratch_err[MAX_DEVICES];

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device, with that device current).
static cor_status scratch_of(int dev, void** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(COR_E_DEVICE, "device index out of range");
    std::call_once(g_scratch_once[dev], [dev] {
        void* p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch[dev])
        return hip_fail(g_scratch_err[dev] != hipSuccess ? g_scratch_err[dev] : hipErrorUnknown,
                        "hipGetSymbolAddress(scratch)");
    *out = g_scratch[dev];
    return COR_OK;
}

}  // namespace cor

using namespace cor;

extern "C" cor_status cor_utv_ex_noalloc(const cor_problem* prob, const cor_opts* opts,
                                         cor_info* info, void* stream) {
    if (!prob) return fail(COR_E_INVAL, "null problem");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void* mem = nullptr;
    cor_status st = scratch_of(dev, &mem);
    if (st != COR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // Calls on one device share its array: one at a time within the process.
    std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
    Plan* P = nullptr;
    st = plan_create(prob, 1, opts, &P, s, false, mem, COR_NOALLOC_SCRATCH_BYTES);
    if (st != COR_OK) return st;
    st = plan_run(P, s);
    // plan_info waits for the stream (also after a failed launch), so the
    // array is idle when the lock is released.
    const cor_status st_info = plan_info(P, info, s);
    if (st == COR_OK) st = st_info;
    if (info) info->device_ms = 0.0;
    plan_destroy(P, s);
    return st;
}
