// Host-side helpers shared by the C ABI units (validation, launch timing,
// workspace arithmetic).  Host code only.
#pragma once

#include <cstddef>
#include <cstdint>

#include "common.h"

namespace prenom {
namespace host {

prenom_status fail(prenom_status st, const char* fmt, ...);
const char* last_error();  // the calling thread's last message
prenom_status hip_status(hipError_t e, const char* what);

// Kernel timing: when profiling is on, a pair of pooled events (else false).
bool prof_events(hipEvent_t* a, hipEvent_t* b);
void prof_record(const char* name, hipEvent_t a, hipEvent_t b);

// Runs one launcher; brackets it with events when timing is on.
template <class F>
hipError_t timed(const char* name, hipStream_t s, F&& launch)
{
    hipEvent_t a = nullptr, b = nullptr;
    const bool on = prof_events(&a, &b);
    if (on) hipEventRecord(a, s);
    const hipError_t e = launch();
    if (on) {
        hipEventRecord(b, s);
        prof_record(name, a, b);
    }
    return e;
}

inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

int device_cus();  // compute units of the current device
prenom_status check_arch(const prenom_arch* a);
prenom_status check_supported(const prenom_arch* a);
MlpShape mlp_shape(const prenom_arch* a);
hipError_t mlp_fwd_any(const MlpShape& m, const float* w, const float* y, int64_t n_s, float* sc, float* act,
                       hipStream_t s);
hipError_t mlp_bwd_any(const MlpShape& m, const float* w, const float* y, const float* dout, const float* sc,
                       int64_t n_s, float* dy, float* partial, float* act, hipStream_t s);
int64_t table_params(const prenom_arch* a);
int64_t mlp_params(const prenom_arch* a);
int64_t mlp_params_of(const MlpShape& m);
GridInfo grid_info(const prenom_arch* a);
prenom_status check_sample_cfg(const prenom_sample_cfg* cfg, bool need_prior_fields);
prenom_status check_render_cfg(const prenom_render_cfg* cfg);
prenom_status check_model(const prenom_model* m, bool need_grads);
// Prior refresh of R^3 vertices in chunks of `chunk`: features into y
// ([L][chunk][2]), head outputs into sc ([chunk][4]), densities into prior_out.
prenom_status prior_refresh_chunks(const prenom_model* model, int32_t R, float* prior_out, float* y, float* sc,
                                   int64_t chunk, hipStream_t s);

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

template <typename T>
T* at(void* base, size_t off)
{
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

}  // namespace host
}  // namespace prenom

#define PRENOM_TRY_HIP(expr, what)                                  \
    do {                                                            \
        const prenom_status st_ = ::prenom::host::hip_status((expr), what); \
        if (st_ != PRENOM_OK) return st_;                           \
    } while (0)

#define PRENOM_LAUNCH(name, stream, expr) \
    PRENOM_TRY_HIP(::prenom::host::timed(name, stream, [&] { return (expr); }), name)
