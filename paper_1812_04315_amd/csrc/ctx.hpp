// Library context and host helpers shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "internal.hpp"

using namespace cnmf;

struct cnmf_ctx {
    Dev dev;
    Control* ctl = nullptr;       // device
    uint64_t* slots = nullptr;    // device, tagged exchange words of the phase kernels
    uint64_t* oxch = nullptr;     // device, tagged exchange words of the orthonormalisation
    float* beta = nullptr;        // device, momentum weights (kBetaLen)
    unsigned seq = 0;             // last tag used
    int dlag = -1;                // stop-test lag (-1: automatic, see the phase launcher)
    char* ws = nullptr;           // device workspace
    size_t ws_bytes = 0;
    char* scratch = nullptr;      // device address of this device's no-alloc scratch
    double clock_hz = 1e8;
};


inline int from_hip(hipError_t e) { return e == hipSuccess ? CNMF_OK : CNMF_EHIP; }

// Tag of the next phase launch; tags are 22 bits, so the words are cleared
// whenever the sequence wraps and no stale word can ever match.
inline hipError_t next_seq(cnmf_ctx* c, unsigned* seq) {
    if (++c->seq >= (1u << 22)) {
        hipError_t e = fill_u64(c->dev, c->slots, (int64_t)kSlotWords, 0);
        if (e != hipSuccess) return e;
        e = fill_u64(c->dev, c->oxch, (int64_t)orth_exchange_words(), 0);
        if (e != hipSuccess) return e;
        c->seq = 1;
    }
    *seq = c->seq;
    return hipSuccess;
}

// count consecutive sequence numbers for the phases of one launch; base
// receives the first
inline hipError_t reserve_seq(cnmf_ctx* c, unsigned count, unsigned* base) {
    if (c->seq + count + 1 >= (1u << 22)) {
        hipError_t e = fill_u64(c->dev, c->slots, (int64_t)kSlotWords, 0);
        if (e != hipSuccess) return e;
        e = fill_u64(c->dev, c->oxch, (int64_t)orth_exchange_words(), 0);
        if (e != hipSuccess) return e;
        c->seq = 0;
    }
    *base = c->seq + 1;
    c->seq += count;
    return hipSuccess;
}

#define CK(x)                                   \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return CNMF_EHIP; \
    } while (0)

// Bump allocator over the context workspace; sizes are rounded to 256 B.
struct Arena {
    size_t off = 0;
    template <class T>
    size_t take(size_t count) {
        size_t at = off;
        off += (count * sizeof(T) + 255) & ~size_t(255);
        return at;
    }
};

inline int ensure_ws(cnmf_ctx* c, size_t bytes) {
    if (bytes <= c->ws_bytes) return CNMF_OK;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    if (c->ws) {
        if (hipStreamSynchronize(c->dev.stream) != hipSuccess) return CNMF_EHIP;
        (void)hipFree(c->ws);
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    if (hipMalloc((void**)&c->ws, want) != hipSuccess) {
        c->ws = nullptr;
        return CNMF_ENOMEM;
    }
    c->ws_bytes = want;
    return CNMF_OK;
}

template <class T>
inline T* at(cnmf_ctx* c, size_t off) { return reinterpret_cast<T*>(c->ws + off); }

inline bool bad_ptr(const void* p) { return p == nullptr; }

inline int check_params(const cnmf_params* prm, int64_t n, int64_t m, bool need_ell) {
    if (!prm) return CNMF_EINVAL;
    if (prm->p < 1 || prm->p > CNMF_MAX_RANK) return CNMF_EINVAL;
    if (prm->reserved != 0) return CNMF_EINVAL;
    if (need_ell) {
        const int64_t l = (int64_t)prm->p + prm->nu;
        if (prm->nu < 0 || l > CNMF_MAX_RANK || l > n || l > m) return CNMF_EINVAL;
        if (prm->q < 1) return CNMF_EINVAL;
        if (!(prm->tau2 > 0.0 && prm->tau2 < 1.0)) return CNMF_EINVAL;
    }
    if (prm->outer_iters < 0 || prm->inner_max < 1 || prm->inner_max > 100000) return CNMF_EINVAL;
    if (prm->inner_min < 1) return CNMF_EINVAL;
    if (!(prm->inner_ratio >= 0.0)) return CNMF_EINVAL;
    if (prm->stop_rule != CNMF_STOP_GLOBAL && prm->stop_rule != CNMF_STOP_SUBPROBLEM)
        return CNMF_EINVAL;
    if (prm->sweep_prec != CNMF_PREC_FP32 && prm->sweep_prec != CNMF_PREC_BF16) return CNMF_EINVAL;
    if (prm->solver != CNMF_SOLVER_NESTEROV && prm->solver != CNMF_SOLVER_HALS &&
        prm->solver != CNMF_SOLVER_MU)
        return CNMF_EINVAL;
    if (prm->restart != CNMF_RESTART_NONE && prm->restart != CNMF_RESTART_GRADIENT) return CNMF_EINVAL;
    if (prm->restart != CNMF_RESTART_NONE && prm->solver != CNMF_SOLVER_NESTEROV) return CNMF_EINVAL;
    if (!(prm->time_budget >= 0.0) || prm->time_budget > 1e6) return CNMF_EINVAL;
    return CNMF_OK;
}


// Algorithm 2 for one instance (api.hip); Xb non-null selects the BF16 sweeps.
int rsi_run(cnmf_ctx* c, int64_t n, int64_t m, const float* X, const uint16_t* Xb, int64_t ldx,
            const cnmf_params* prm, const float* oL, const float* oR, float* QL_out,
            float* QR_out, float* XL_out, float* XR_out);
