// Allocation-free prior refresh: prenom_prior_refresh with its workspace (the
// per-vertex features and head outputs of one chunk) in a fixed device array
// of this library instead of a caller buffer.  Host code plus one __device__
// array; the kernels are those of prenom_prior_refresh.
#include <mutex>

#include "api_util.h"
#include "common.h"

namespace {

using namespace prenom;
using namespace prenom::host;

constexpr size_t kScratchBytes = PRENOM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, at its own address.  In host code this name is only a
// stand-in for the symbol: the device address comes from hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array; looked up once per
// device (with that device current) and kept.
prenom_status scratch_of_current_device(void** out)
{
    int dev = 0;
    PRENOM_TRY_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PRENOM_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        PRENOM_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(PRENOM_ERR_HIP, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PRENOM_OK;
}

// Largest chunk (a multiple of 1024 vertices) whose features and head outputs
// fit the scratch array; 0 if not even 1024 fit.
int64_t noalloc_chunk(const prenom_arch* a)
{
    const size_t per = (size_t)a->n_levels * (size_t)a->n_features * sizeof(float);
    int64_t c = (int64_t)((kScratchBytes - 2 * kAlign) / (per + 4 * sizeof(float))) / 1024 * 1024;
    while (c > 0 && align_up((size_t)c * per) + align_up((size_t)c * 4 * sizeof(float)) > kScratchBytes) c -= 1024;
    return c;
}

}  // namespace

extern "C" {

size_t prenom_noalloc_scratch_bytes(void) { return kScratchBytes; }

prenom_status prenom_prior_refresh_noalloc(const prenom_model* model, int32_t R, float* prior_out, void* stream)
{
    prenom_status st = check_model(model, false);
    if (st != PRENOM_OK) return st;
    if (R < 2 || R > PRENOM_MAX_PRIOR_RES) return fail(PRENOM_ERR_SHAPE, "R %d outside [2, %d]", R, PRENOM_MAX_PRIOR_RES);
    if (!prior_out) return fail(PRENOM_ERR_INVALID_ARG, "prior_out is NULL");
    const int64_t chunk = noalloc_chunk(&model->arch);
    if (chunk < 1024)
        return fail(PRENOM_ERR_WORKSPACE, "%d levels x %d features do not fit the %zu-byte scratch array",
                    model->arch.n_levels, model->arch.n_features, kScratchBytes);
    void* base = nullptr;
    st = scratch_of_current_device(&base);
    if (st != PRENOM_OK) return st;
    const size_t per = (size_t)model->arch.n_levels * (size_t)model->arch.n_features * sizeof(float);
    float* y = at<float>(base, 0);
    float* sc = at<float>(base, align_up((size_t)chunk * per));
    return prior_refresh_chunks(model, R, prior_out, y, sc, chunk, (hipStream_t)stream);
}

}  // extern "C"
