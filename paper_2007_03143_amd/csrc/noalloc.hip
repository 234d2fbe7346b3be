// Integration of a built context with its per-integration device scratch in
// a static device array, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc). The kernels are those of xc_context_integrate; only the memory
// they use for the wave scratch, the tile map and the request descriptor
// differs.
#include <mutex>

#include "xc_internal.hpp"

namespace xc {

constexpr size_t kStaticScratchBytes = XC_STATIC_SCRATCH_BYTES;
constexpr size_t kReqBytes = 256;     // room for the request descriptor
constexpr int kMaxDevices = 64;
static_assert(sizeof(ReqDev) <= kReqBytes, "request descriptor fits its slot");

// One copy per GPU, held until the process ends. Host code never takes the
// address of this name: on the host it is a stand-in symbol, not a device
// address. The device address of each GPU's copy comes from
// hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) char scratch[kStaticScratchBytes];

static std::mutex g_static_mu;
static char* g_static_ptr[kMaxDevices] = {};

// Device address of the current device's copy of the array, looked up once
// per device (with that device current) and kept.
static int static_scratch(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(XC_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(static scratch)");
        if (!p) return fail(XC_ERR_DEVICE, "hipGetSymbolAddress returned a null address");
        g_static_ptr[dev] = (char*)p;
    }
    *out = g_static_ptr[dev];
    return XC_OK;
}

static size_t round256(size_t n) { return (n + 255) / 256 * 256; }

int run_integrate_noalloc(xc_context* c, int functional, int precision, const double* dP,
                          double* dV, double* dEN) {
    int dev = 0;
    XC_HIP(hipGetDevice(&dev));
    if (dev != c->device)
        return fail(XC_ERR_STATE, "the context's device is not the current device");
    // layout: request descriptor | tile map of the largest wave | (split-BF16
    // mode) digits and row scales of P | wave scratch
    const bool bf16 = precision == XC_MIXED_BF16;
    const size_t tmap_bytes = round256(2 * sizeof(int) * (size_t)c->max_tiles);
    const size_t dig_bytes = bf16 ? round256(8 * (size_t)c->nbf * c->nbf) : 0;
    const size_t scl_bytes = bf16 ? round256(8 * (size_t)c->nbf) : 0;
    const size_t need = kReqBytes + tmap_bytes + dig_bytes + scl_bytes + c->max_wave_bytes;
    if (need > kStaticScratchBytes)
        return fail(XC_ERR_NOMEM,
                    "the context's largest wave needs " + std::to_string(need) +
                        " bytes of scratch, above the static maximum of " +
                        std::to_string(kStaticScratchBytes) +
                        " (create the context with a smaller wave_bytes)");
    char* base = nullptr;
    XC_TRY(static_scratch(dev, &base));
    ReqDev* d_req = (ReqDev*)base;
    int* d_tmap = (int*)(base + kReqBytes);
    unsigned long long* d_dig = (unsigned long long*)(base + kReqBytes + tmap_bytes);
    double* d_scl = (double*)(base + kReqBytes + tmap_bytes + dig_bytes);
    char* wave_scratch = base + kReqBytes + tmap_bytes + dig_bytes + scl_bytes;

    const bool gga = functional == XC_GGA_PBE;
    XC_TRY(launch_fill(c->stream, dV, (long long)c->nbf * c->nbf, 0.0));
    ReqDev req = make_req(c, dP, dV);
    if (bf16) {
        XC_TRY(launch_p_digits(c->stream, dP, c->nbf, d_dig, d_scl));
        req.Pdig = d_dig;
        req.Pscale = d_scl;
    }
    XC_TRY(launch_put_req(c->stream, d_req, req));
    const WaveBatch* wb = (const WaveBatch*)c->d_wb.p;
    const int* gpre = (const int*)c->d_gemm_pre.p;
    const int* spre = (const int*)c->d_syr_pre.p;
    const int* wpre = (const int*)c->d_wide_pre.p;
    for (const Wave& w : c->waves)
        XC_TRY(launch_wave(nullptr, c->stream, gga, precision, wb + w.wb_off, gpre + w.pre_off,
                           spre + w.pre_off, wpre + w.pre_off, w.count, w.gemm_tiles,
                           w.syr_tiles, w.wide_tiles, w.wide, d_req, wave_scratch, d_tmap, true,
                           c->any_pure));
    return launch_finish(nullptr, c->stream, dV, c->nbf, (const double*)c->epart.p,
                         (const double*)c->npart.p, c->n_batches, dEN);
}

}  // namespace xc
