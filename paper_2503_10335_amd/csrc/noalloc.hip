// tbsci_sigma_noalloc: the sigma build with its only scratch buffer -- the
// beta sweep's transposed block of C and its sweep result -- in a
// file-scope device array instead of memory the library allocates, for
// callers that cannot allocate (code under stream capture, serving loops
// that forbid it).  The array is per device: each GPU the library runs on
// holds its own copy until the process ends, and host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
#include <mutex>

#include "tbsci_internal.hpp"

namespace tbsci {
namespace {

// 64 MiB: the beta sweep of every alpha row of a space with l_beta up to
// 4.19e6 strings fits in blocks of at least one row
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// device address of this device's scratch array (device current)
void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) throw Error(TBSCI_E_INVAL, "device index too large");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw Error(TBSCI_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                            hipGetErrorString(e));
        g_ptr[device] = p;
    }
    return g_ptr[device];
}

}  // namespace
}  // namespace tbsci

using namespace tbsci;

extern "C" {

int tbsci_sigma_noalloc(tbsci_ctx *ctx, const void *C_dev, void *sigma_dev, int precision,
                        void *stream) {
    return guarded([&]() -> int {
        check_ctx(ctx);  // makes the context's device current
        Ctx *c = ctx_of(ctx);
        if (precision != TBSCI_FP64 && precision != TBSCI_FP32)
            throw Error(TBSCI_E_INVAL, "precision must be TBSCI_FP64 or TBSCI_FP32");
        check_dev(C_dev, c->device, "C");
        check_dev(sigma_dev, c->device, "sigma");
        if (C_dev == sigma_dev) throw Error(TBSCI_E_INVAL, "C and sigma must not alias");
        if (c->dets)
            throw Error(TBSCI_E_INVAL, "tbsci_sigma_noalloc takes whole TPB spaces only (a "
                                       "TBSCI space needs two zero-extended vectors)");
        if (beta_block_rows(c->sp[0].l, c->sp[1].l, kScratchBytes) < 1)
            throw Error(TBSCI_E_INVAL, "l_beta exceeds what the 64 MiB static workspace of "
                                       "tbsci_sigma_noalloc holds (4.19e6 strings)");
        void *w = scratch_ptr(c->device);
        launch_sigma_ws(*c, C_dev, sigma_dev, precision, (hipStream_t)stream, 7, w,
                        kScratchBytes, false);
        return TBSCI_OK;
    });
}

}  // extern "C"
