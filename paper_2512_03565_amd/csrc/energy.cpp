// energy.cpp -- the GPU's energy counter, for energy as a tuning metric
// (section 2.3.3: the tuner may minimise energy instead of runtime; section
// 5's Benchmark B compares the two optima).
//
// The board's energy accumulator is read through AMD SMI (libamd_smi, loaded
// on first use, so the library itself does not depend on it).  The firmware
// refreshes the accumulator about once a second; each refresh carries a
// timestamp in nanoseconds, and counts convert to joules by the counter's
// resolution (microjoules per count).
#include <dlfcn.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include <amd_smi/amdsmi.h>

#include "internal.h"

namespace {

struct Smi {
    bool tried = false, ok = false;
    void *so = nullptr;
    amdsmi_status_t (*init)(uint64_t) = nullptr;
    amdsmi_status_t (*from_bdf)(amdsmi_bdf_t, amdsmi_processor_handle *) = nullptr;
    amdsmi_status_t (*energy)(amdsmi_processor_handle, uint64_t *, float *, uint64_t *) = nullptr;
    amdsmi_processor_handle dev[64] = {};
    std::string why;
};

Smi g_smi;
std::mutex g_smi_mu;

bool smi_load(Smi &s)
{
    if (s.tried) return s.ok;
    s.tried = true;
    const char *names[] = {"libamd_smi.so", "libamd_smi.so.26", "/opt/rocm/lib/libamd_smi.so"};
    for (const char *n : names)
        if ((s.so = dlopen(n, RTLD_NOW | RTLD_LOCAL)) != nullptr) break;
    if (!s.so) {
        s.why = "AMD SMI library not found";
        return false;
    }
    s.init = (amdsmi_status_t(*)(uint64_t))dlsym(s.so, "amdsmi_init");
    s.from_bdf = (amdsmi_status_t(*)(amdsmi_bdf_t, amdsmi_processor_handle *))dlsym(
        s.so, "amdsmi_get_processor_handle_from_bdf");
    s.energy = (amdsmi_status_t(*)(amdsmi_processor_handle, uint64_t *, float *, uint64_t *))dlsym(
        s.so, "amdsmi_get_energy_count");
    if (!s.init || !s.from_bdf || !s.energy) {
        s.why = "AMD SMI library lacks the energy-counter calls";
        return false;
    }
    if (s.init(AMDSMI_INIT_AMD_GPUS) != AMDSMI_STATUS_SUCCESS) {
        s.why = "amdsmi_init failed";
        return false;
    }
    s.ok = true;
    return true;
}

}  // namespace

// AMD SMI handle of the current HIP device (found by its PCI address).
static mdlj_status smi_device(mdlj_ctx *ctx, amdsmi_processor_handle *h)
{
    int dev = -1;
    HIPCHK(ctx, hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_smi_mu);
    if (!smi_load(g_smi)) return set_err(ctx, MDLJ_ERR_NOTFOUND, g_smi.why);
    if (dev < 0 || dev >= 64) return set_err(ctx, MDLJ_ERR_ARG, "device index beyond the table");
    if (!g_smi.dev[dev]) {
        char bus[64] = {0};
        HIPCHK(ctx, hipDeviceGetPCIBusId(bus, (int)sizeof bus, dev));
        unsigned dom = 0, b = 0, d = 0, f = 0;
        if (sscanf(bus, "%x:%x:%x.%x", &dom, &b, &d, &f) != 4)
            return set_err(ctx, MDLJ_ERR_HIP, std::string("unreadable PCI address ") + bus);
        amdsmi_bdf_t bdf;
        bdf.as_uint = 0;
        bdf.domain_number = dom;
        bdf.bus_number = b;
        bdf.device_number = d;
        bdf.function_number = f;
        amdsmi_processor_handle p = nullptr;
        if (g_smi.from_bdf(bdf, &p) != AMDSMI_STATUS_SUCCESS || !p)
            return set_err(ctx, MDLJ_ERR_NOTFOUND, std::string("no AMD SMI device at ") + bus);
        g_smi.dev[dev] = p;
    }
    *h = g_smi.dev[dev];
    return MDLJ_OK;
}

mdlj_status energy_read(mdlj_ctx *ctx, double *joules, uint64_t *ts_ns)
{
    amdsmi_processor_handle h = nullptr;
    STCHK(smi_device(ctx, &h));
    uint64_t acc = 0, ts = 0;
    float res = 0.0f;
    if (g_smi.energy(h, &acc, &res, &ts) != AMDSMI_STATUS_SUCCESS)
        return set_err(ctx, MDLJ_ERR_NOTFOUND, "energy counter not readable");
    *joules = (double)acc * (double)res * 1e-6;
    *ts_ns = ts;
    return MDLJ_OK;
}

extern "C" {

mdlj_status mdlj_gpu_energy(mdlj_ctx *ctx, double *joules, double *seconds)
{
    if (!ctx || !joules || !seconds) return MDLJ_ERR_ARG;
    uint64_t ts = 0;
    STCHK(energy_read(ctx, joules, &ts));
    *seconds = (double)ts * 1e-9;
    return MDLJ_OK;
}

}  // extern "C"
