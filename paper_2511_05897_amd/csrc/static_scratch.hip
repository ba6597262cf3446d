// The assembled ladder (sum_Q B^Q Z B^Q, eq 25 inserted into the ladder term) for callers that
// cannot allocate device memory: its scratch (the reduced-precision copies of the operands and the
// intermediate V) lives in one file-scope device array per GPU instead of a caller workspace.
//
// The array's name is a host-side stand-in in host code; its device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and only that address is passed on.
// Every call on a GPU shares that GPU's array: calls that overlap on one GPU (two streams, two host
// threads) race on it.  Nothing in it has to start at zero: the first step of every auxiliary
// chunk overwrites V, and the rounded copies are rewritten by every call.
#include "internal.h"
#include "../../include/adc3ea.h"

#include <mutex>
#include <string>

namespace adc3 {
namespace {

static __device__ __align__(256) unsigned char scratch[ADC3_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of this device's copy of the scratch array (looked up on the first call per device)
void* scratch_ptr() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(ADC3_EUNSUP, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(ADC3_EHIP, "hipGetSymbolAddress returned no address for the static scratch");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace adc3

using namespace adc3;

extern "C" int adc3_ladder_apply_static(const double* Bvv, const double* Z, double* C, int nvir, int naux,
                                        int nrows, int precision, hipStream_t stream) {
    try {
        if (nvir <= 0 || naux < 0 || nrows <= 0) fail(ADC3_EINVAL, "nvir and nrows must be > 0 and naux >= 0");
        if (nvir > 1024 || nrows > 65535) fail(ADC3_EINVAL, "nvir > 1024 or nrows > 65535 is not supported");
        if (precision < 0 || precision > 2) fail(ADC3_EINVAL, "precision must be 0, 1 or 2");
        if (!Bvv || !Z || !C) fail(ADC3_EINVAL, "NULL pointer argument");
        const size_t need = adc3_ladder_workspace_bytes(nvir, naux, nrows, precision);
        if (need > (size_t)ADC3_STATIC_SCRATCH_BYTES)
            fail(ADC3_ENOMEM, "shape needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                                  std::to_string((size_t)ADC3_STATIC_SCRATCH_BYTES));
        char* base = (char*)scratch_ptr();
        const long long vv = (long long)nvir * nvir;
        const size_t eb = precision == 0 ? 8 : precision == 1 ? 4 : 2;
        const void *Bp = Bvv, *Zp = Z;
        size_t off = 0;
        if (precision > 0) {
            void* Bl = base;
            off = ((size_t)naux * vv * eb + 255) & ~size_t(255);
            void* Zl = base + off;
            off += ((size_t)nrows * vv * eb + 255) & ~size_t(255);
            k_to_lowp(Bl, Bvv, (long long)naux * vv, precision, stream);
            k_to_lowp(Zl, Z, nrows * vv, precision, stream);
            Bp = Bl;
            Zp = Zl;
        }
        // the rest of the array holds the intermediate: as many auxiliary functions per chunk as fit
        const long long ve = (long long)(((size_t)ADC3_STATIC_SCRATCH_BYTES - off) / eb);
        df_ladder(precision, nrows, nvir, naux, Bp, Zp, C, false, base + off, ve, stream);
        return ADC3_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::exception& e) {
        set_error(e.what());
        return ADC3_EINVAL;
    }
}
