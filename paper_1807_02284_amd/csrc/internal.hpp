// internal.hpp -- declarations shared by the translation units of libcslbm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/cslbm.h"
#include "cm_collide.hpp"

namespace cslbm {

// error reporting: fail() records a thread-local message and returns code
int fail(int code, const char* fmt, ...);
int check_launch(const char* what);

#define CSLBM_HIP_TRY(call)                                                                      \
    do {                                                                                         \
        const hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return ::cslbm::fail(CSLBM_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// storage traits: FP32 or IEEE binary16 shifted populations
template <typename T>
struct Io;

template <>
struct Io<float> {
    static __device__ __forceinline__ float ld(const float* p) { return *p; }
    static __device__ __forceinline__ void st(float* p, float v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Io<_Float16> {
    static __device__ __forceinline__ float ld(const _Float16* p) { return static_cast<float>(*p); }
    static __device__ __forceinline__ void st(_Float16* p, float v)
    {
        __builtin_nontemporal_store(static_cast<_Float16>(v), p);   // round to nearest even
    }
};

int64_t cells_of(const cslbm_level* L);
int validate_shape(const cslbm_level* L);
int validate_params(const cslbm_level* L);
Rates make_rates(const cslbm_params& p);

// Thread block for the one-thread-per-cell kernels over an nx-wide row.
dim3 step_block(int nx);

// One collide-stream step of level L from (fin, gin) into (fout, gout);
// L's own f/g pointers are not used.  Arguments must be validated.
int launch_step_into(const cslbm_level* L, const void* fin, void* fout, const float* gin,
                     float* gout, hipStream_t stream);

// One step in the finite-difference gradient mode (grad_mode 1): the
// adaptive factor takes |grad u|_F of vel, the input state's velocity, and
// the new state's velocity goes to vel_out.  With gmax_running the field
// maximum of that gradient is reduced into L->gmax_buf first.
int launch_step_grad(const cslbm_level* L, const void* fin, void* fout, const float* gin,
                     float* gout, const float* vel, float* vel_out, hipStream_t stream);

// The same step with its output replaced by the quadratic time interpolation
// l0 * t0 + l1 * fin + l2 * step(fin) at every cell (and likewise for g);
// L must have flags.
int launch_step_interp(const cslbm_level* L, const void* fin, void* fout, const float* gin,
                       float* gout, const void* t0, const float* gt0, double l0, double l1,
                       double l2, hipStream_t stream);

// Time weight between a parent's states at t_n (0) and t_n + dt_0 (1) of the
// prior-mapping before sub-step k = 1..l of a finer scale with spacing ratio
// alpha (section "Temporal alignment and scale mapping"): the first l - 1
// sub-steps read the parent blended in time, here at the sub-step's start
// time (k - 1) dt_f; the final sub-step reads the parent at t_n + dt_0.
inline double prior_weight(int k, int l, double alpha) { return k == l ? 1.0 : (k - 1) / alpha; }

}  // namespace cslbm
