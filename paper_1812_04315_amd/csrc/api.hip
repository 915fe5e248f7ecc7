// C ABI of libcnmf: argument validation, workspace, and the enqueue order of
// randomized subspace iteration (Sec. 3, Algorithm 2) and of the plain and
// compressed NeNMF outer loops (Sec. 2; Sec. 3, Algorithm 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>

#include "internal.hpp"

using namespace cnmf;

struct cnmf_ctx {
    Dev dev;
    Control* ctl = nullptr;       // device
    char* ws = nullptr;           // device workspace
    size_t ws_bytes = 0;
    double clock_hz = 1e8;
};

namespace {

int from_hip(hipError_t e) { return e == hipSuccess ? CNMF_OK : CNMF_EHIP; }

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

int ensure_ws(cnmf_ctx* c, size_t bytes) {
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
T* at(cnmf_ctx* c, size_t off) { return reinterpret_cast<T*>(c->ws + off); }

bool bad_ptr(const void* p) { return p == nullptr; }

int check_params(const cnmf_params* prm, int64_t n, int64_t m, bool need_ell) {
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
    return CNMF_OK;
}

}  // namespace

extern "C" {

void cnmf_params_default(cnmf_params* out) {
    if (!out) return;
    std::memset(out, 0, sizeof(*out));
    out->p = 0;
    out->nu = 10;
    out->q = 4;
    out->outer_iters = 200;
    out->inner_max = 500;
    out->inner_min = 1;
    out->inner_ratio = 1e-3;
    out->tau2 = 1e-9;
    out->stop_rule = CNMF_STOP_GLOBAL;
    out->sweep_prec = CNMF_PREC_FP32;
    out->flags = 0;
}

const char* cnmf_strerror(int code) {
    switch (code) {
        case CNMF_OK: return "ok";
        case CNMF_EINVAL: return "invalid argument";
        case CNMF_ENOMEM: return "out of device memory";
        case CNMF_EHIP: return "HIP runtime error";
        case CNMF_EDEVICE: return "device reported an error (see status word)";
        default: return "unknown error";
    }
}

int cnmf_create(cnmf_ctx** out, int device, void* stream) {
    if (!out) return CNMF_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return CNMF_EHIP;
    if (device < 0 || device >= count) return CNMF_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return CNMF_EHIP;
    cnmf_ctx* c = new (std::nothrow) cnmf_ctx();
    if (!c) return CNMF_ENOMEM;
    c->dev.device = device;
    c->dev.stream = (hipStream_t)stream;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0) {
        delete c;
        return CNMF_EHIP;
    }
    c->dev.num_cus = cus;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        c->clock_hz = 1000.0 * khz;
    if (hipMalloc((void**)&c->ctl, sizeof(Control)) != hipSuccess) {
        delete c;
        return CNMF_ENOMEM;
    }
    if (hipMemset(c->ctl, 0, sizeof(Control)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->ctl);
        delete c;
        return CNMF_EHIP;
    }
    *out = c;
    return CNMF_OK;
}

int cnmf_destroy(cnmf_ctx* c) {
    if (!c) return CNMF_EINVAL;
    (void)hipSetDevice(c->dev.device);
    (void)hipStreamSynchronize(c->dev.stream);
    if (c->ws) (void)hipFree(c->ws);
    if (c->ctl) (void)hipFree(c->ctl);
    delete c;
    return CNMF_OK;
}

int cnmf_set_stream(cnmf_ctx* c, void* stream) {
    if (!c) return CNMF_EINVAL;
    c->dev.stream = (hipStream_t)stream;
    return CNMF_OK;
}

int cnmf_clock_hz(cnmf_ctx* c, double* hz) {
    if (!c || !hz) return CNMF_EINVAL;
    *hz = c->clock_hz;
    return CNMF_OK;
}

int cnmf_status(cnmf_ctx* c, int32_t* status) {
    if (!c || !status) return CNMF_EINVAL;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    if (hipStreamSynchronize(c->dev.stream) != hipSuccess) return CNMF_EHIP;
    Control h;
    if (hipMemcpy(&h, c->ctl, sizeof(Control), hipMemcpyDeviceToHost) != hipSuccess) return CNMF_EHIP;
    *status = h.status;
    // Clear the word; after a stalled barrier also reset the barrier state.
    Control z = h;
    z.status = 0;
    if (h.status & CNMF_ST_TIMEOUT) {
        z.bar_count = 0;
    }
    if (hipMemcpy(c->ctl, &z, sizeof(Control), hipMemcpyHostToDevice) != hipSuccess) return CNMF_EHIP;
    return (h.status & ~CNMF_ST_ZERO_LIPS) ? CNMF_EDEVICE : CNMF_OK;
}

// ---------------------------------------------------------------------------
// Kernel-level entry points
// ---------------------------------------------------------------------------

int cnmf_sweep_right(cnmf_ctx* c, int64_t R, int64_t C, const float* X, int64_t ldx, int32_t k,
                     const float* A, int64_t lda, int32_t a_trans, float* Y, int64_t ldy) {
    if (!c || R < 0 || C < 0 || k < 1 || k > 32) return CNMF_EINVAL;
    if (R == 0) return CNMF_OK;
    if (bad_ptr(Y) || ldy < k) return CNMF_EINVAL;
    if (C > 0 && (bad_ptr(X) || bad_ptr(A) || ldx < C)) return CNMF_EINVAL;
    if (C > 0 && (a_trans ? lda < C : lda < k)) return CNMF_EINVAL;
    if (C == 0) {  // empty reduction: Y = 0
        if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
        return from_hip(hipMemset2DAsync(Y, ldy * sizeof(float), 0, k * sizeof(float), R,
                                         c->dev.stream));
    }
    Arena a;
    size_t off = a.take<float>(sweep_right_partial_floats(c->dev, R, C));
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    return from_hip(sweep_right(c->dev, R, C, X, ldx, k, A, lda, a_trans != 0, Y, ldy,
                                at<float>(c, off)));
}

int cnmf_sweep_left(cnmf_ctx* c, int64_t R, int64_t C, const float* X, int64_t ldx, int32_t k,
                    const float* B, int64_t ldb, float* Z, int64_t ldz, int32_t z_trans) {
    if (!c || R < 0 || C < 0 || k < 1 || k > 32) return CNMF_EINVAL;
    if (C == 0) return CNMF_OK;
    if (bad_ptr(Z) || (z_trans ? ldz < C : ldz < k)) return CNMF_EINVAL;
    if (R > 0 && (bad_ptr(X) || bad_ptr(B) || ldx < C || ldb < k)) return CNMF_EINVAL;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    if (R == 0) {
        if (z_trans)
            return from_hip(hipMemset2DAsync(Z, ldz * sizeof(float), 0, C * sizeof(float), k,
                                             c->dev.stream));
        return from_hip(hipMemset2DAsync(Z, ldz * sizeof(float), 0, k * sizeof(float), C,
                                         c->dev.stream));
    }
    Arena a;
    size_t off = a.take<float>(sweep_left_partial_floats(c->dev, R, C));
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    return from_hip(sweep_left(c->dev, R, C, X, ldx, k, B, ldb, Z, ldz, z_trans != 0,
                               at<float>(c, off)));
}

int cnmf_orth(cnmf_ctx* c, int64_t N, int32_t l, const float* Y, const float* pool,
              int32_t pool_trans, double tau2, float* Q, int32_t* replaced) {
    if (!c || N < 1 || l < 1 || l > 32 || l > N) return CNMF_EINVAL;
    if (bad_ptr(Y) || bad_ptr(pool) || bad_ptr(Q)) return CNMF_EINVAL;
    if (!(tau2 > 0.0 && tau2 < 1.0)) return CNMF_EINVAL;
    Arena a;
    size_t off = a.take<double>(orth_workspace_doubles(c->dev, N, l));
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    return from_hip(orth(c->dev, N, l, Y, pool, pool_trans != 0, tau2, Q, replaced,
                         at<double>(c, off), c->ctl));
}

int cnmf_lipschitz(cnmf_ctx* c, int32_t p, const float* W, double* out) {
    if (!c || p < 1 || p > 32 || bad_ptr(W) || bad_ptr(out)) return CNMF_EINVAL;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    return from_hip(lipschitz(c->dev, p, W, out, c->ctl));
}

int cnmf_nnls(cnmf_ctx* c, int64_t rows, int32_t p, float* Z, int64_t z_rs, int64_t z_cs,
              const float* W, const float* B, double tol, int32_t inner_max, int32_t inner_min,
              int32_t forced, int32_t* steps_out, double* L_out, double* pg2_out) {
    if (!c || rows < 1 || p < 1 || p > 32) return CNMF_EINVAL;
    if (bad_ptr(Z) || bad_ptr(W) || bad_ptr(B)) return CNMF_EINVAL;
    if (inner_max < 1 || inner_max > 100000 || inner_min < 1) return CNMF_EINVAL;
    if ((rows + 255) / 256 > c->dev.num_cus) return CNMF_EINVAL;
    Arena a;
    size_t offL = a.take<double>(1);
    size_t offP = a.take<double>(nnls_partial_doubles(c->dev, rows));
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    double* Ld = at<double>(c, offL);
    CK(lipschitz(c->dev, p, W, Ld, c->ctl));
    NnlsArgs na{};
    na.rows = rows;
    na.p = p;
    na.Z = Z;
    na.z_rs = z_rs;
    na.z_cs = z_cs;
    na.W = W;
    na.B = B;
    na.L = Ld;
    na.tol_value = tol;
    na.inner_max = inner_max;
    na.inner_min = inner_min;
    na.forced = forced;
    na.steps_out = steps_out;
    na.L_out = L_out;
    na.pg2_out = pg2_out;
    return from_hip(nnls(c->dev, na, at<double>(c, offP), c->ctl));
}

// ---------------------------------------------------------------------------
// Randomized subspace iteration (Algorithm 2)
// ---------------------------------------------------------------------------

static int rsi_impl(cnmf_ctx* c, int64_t n, int64_t m, const float* X, const uint16_t* Xb,
                    int64_t ldx, const cnmf_params* prm, const float* oL, const float* oR,
                    float* QL_out, float* QR_out, float* XL_out, float* XR_out) {
    const int l = prm->p + prm->nu;
    const bool bf = Xb != nullptr;
    Arena a;
    const size_t o_oRt = a.take<float>((size_t)n * l);
    const size_t o_Yn = a.take<float>((size_t)n * l);
    const size_t o_QL = a.take<float>((size_t)n * l);
    const size_t o_Ym = a.take<float>((size_t)m * l);
    const size_t o_QRt = a.take<float>((size_t)m * l);
    size_t part = std::max(sweep_right_partial_floats(c->dev, n, m),
                           sweep_left_partial_floats(c->dev, n, m));
    if (bf)
        part = std::max(part, std::max(sweep_right_bf16_partial_floats(c->dev, n, m),
                                       sweep_left_bf16_partial_floats(c->dev, n, m)));
    const size_t o_part = a.take<float>(part);
    const size_t o_orth = a.take<double>(std::max(orth_workspace_doubles(c->dev, n, l),
                                                  orth_workspace_doubles(c->dev, m, l)));
    const size_t o_pk = a.take<uint16_t>(bf ? (size_t)std::max(n, m) * 32 * 2 : 1);
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    const Dev& d = c->dev;
    float* oRt = at<float>(c, o_oRt);
    float* Yn = at<float>(c, o_Yn);
    float* QL = at<float>(c, o_QL);
    float* Ym = at<float>(c, o_Ym);
    float* QRt = at<float>(c, o_QRt);
    float* pt = at<float>(c, o_part);
    double* ows = at<double>(c, o_orth);
    uint16_t* pk = at<uint16_t>(c, o_pk);
    const double tau2 = prm->tau2;

    auto right = [&](const float* A, float* Y) -> hipError_t {   // Y (n x l) = X A, A m x l
        if (bf) return sweep_right_bf16(d, n, m, Xb, ldx, l, A, l, Y, l, pt, pk);
        return sweep_right(d, n, m, X, ldx, l, A, l, false, Y, l, pt);
    };
    auto left = [&](const float* B, float* Z, bool trans) -> hipError_t {  // Z = X^T B
        const int64_t ldz = trans ? m : l;
        if (bf) return sweep_left_bf16(d, n, m, Xb, ldx, l, B, l, Z, ldz, trans, pt, pk);
        return sweep_left(d, n, m, X, ldx, l, B, l, Z, ldz, trans, pt);
    };

    if (!bf && (prm->flags & CNMF_FLAG_VALIDATE_INPUT)) CK(check_input(d, n, m, X, ldx, c->ctl));
    CK(transpose(d, l, n, oR, n, oRt, l));                       // Omega_R^T, n x l
    // Step 0: sketches X Omega_L and (Omega_R X)^T and their bases.
    CK(right(oL, Yn));
    CK(orth(d, n, l, Yn, oRt, false, tau2, QL, nullptr, ows, c->ctl));
    CK(left(oRt, Ym, false));
    CK(orth(d, m, l, Ym, oL, false, tau2, QRt, nullptr, ows, c->ctl));
    for (int k = 1; k <= prm->q; ++k) {
        // Q~_L^(k) = orth(X^T Q_L^(k-1)), kept in the Q_R output (m x l).
        CK(left(QL, Ym, false));
        CK(orth(d, m, l, Ym, oL, false, tau2, QR_out, nullptr, ows, c->ctl));
        // Q~_R^(k)^T = orth(X Q_R^(k-1)^T), kept in the Q_L output (n x l).
        CK(right(QRt, Yn));
        CK(orth(d, n, l, Yn, oRt, false, tau2, QL_out, nullptr, ows, c->ctl));
        // X Q~_L^(k) (n x l) and (Q~_R^(k) X)^T (m x l).
        CK(right(QR_out, XR_out));
        if (k < prm->q) {
            CK(left(QL_out, Ym, false));
            CK(orth(d, n, l, XR_out, oRt, false, tau2, QL, nullptr, ows, c->ctl));
            CK(orth(d, m, l, Ym, oL, false, tau2, QRt, nullptr, ows, c->ctl));
        } else {
            CK(left(QL_out, XL_out, true));   // X_L = Q_L^T X, l x m
        }
    }
    return CNMF_OK;
}

int cnmf_rsi(cnmf_ctx* c, int64_t n, int64_t m, const float* X, int64_t ldx,
             const cnmf_params* prm, const float* omega_L, const float* omega_R, float* Q_L,
             float* Q_R, float* X_L, float* X_R) {
    if (!c || n < 1 || m < 1) return CNMF_EINVAL;
    int rc = check_params(prm, n, m, true);
    if (rc) return rc;
    if (prm->sweep_prec != CNMF_PREC_FP32) return CNMF_EINVAL;
    if (bad_ptr(X) || ldx < m || bad_ptr(omega_L) || bad_ptr(omega_R)) return CNMF_EINVAL;
    if (bad_ptr(Q_L) || bad_ptr(Q_R) || bad_ptr(X_L) || bad_ptr(X_R)) return CNMF_EINVAL;
    return rsi_impl(c, n, m, X, nullptr, ldx, prm, omega_L, omega_R, Q_L, Q_R, X_L, X_R);
}

int cnmf_rsi_bf16(cnmf_ctx* c, int64_t n, int64_t m, const uint16_t* Xb, int64_t ldxb,
                  const cnmf_params* prm, const float* omega_L, const float* omega_R,
                  float* Q_L, float* Q_R, float* X_L, float* X_R) {
    if (!c || n < 1 || m < 1) return CNMF_EINVAL;
    int rc = check_params(prm, n, m, true);
    if (rc) return rc;
    if (bad_ptr(Xb) || ldxb < m || (ldxb % 8) != 0 || (reinterpret_cast<uintptr_t>(Xb) & 15u))
        return CNMF_EINVAL;
    if (bad_ptr(omega_L) || bad_ptr(omega_R)) return CNMF_EINVAL;
    if (bad_ptr(Q_L) || bad_ptr(Q_R) || bad_ptr(X_L) || bad_ptr(X_R)) return CNMF_EINVAL;
    return rsi_impl(c, n, m, nullptr, Xb, ldxb, prm, omega_L, omega_R, Q_L, Q_R, X_L, X_R);
}

int cnmf_to_bf16(cnmf_ctx* c, int64_t n, int64_t m, const float* X, int64_t ldx, uint16_t* Xb,
                 int64_t ldxb) {
    if (!c || n < 0 || m < 0 || bad_ptr(X) || bad_ptr(Xb) || ldx < m || ldxb < m)
        return CNMF_EINVAL;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    return from_hip(to_bf16(c->dev, n, m, X, ldx, Xb, ldxb));
}

// ---------------------------------------------------------------------------
// NeNMF outer loop, plain (Sec. 2) and compressed (Algorithm 1)
// ---------------------------------------------------------------------------

int cnmf_solve(cnmf_ctx* c, int method, int64_t n, int64_t m, const float* X, int64_t ldx,
               const float* Q_L, const float* Q_R, const float* X_L, const float* X_R,
               const cnmf_params* prm, float* G, float* F, const cnmf_trace* trace,
               const int32_t* replay) {
    if (!c || n < 1 || m < 1) return CNMF_EINVAL;
    const bool comp = method == CNMF_METHOD_COMPRESSED;
    if (!comp && method != CNMF_METHOD_PLAIN) return CNMF_EINVAL;
    int rc = check_params(prm, n, m, comp);
    if (rc) return rc;
    if (bad_ptr(G) || bad_ptr(F)) return CNMF_EINVAL;
    if (comp) {
        if (bad_ptr(Q_L) || bad_ptr(Q_R) || bad_ptr(X_L) || bad_ptr(X_R)) return CNMF_EINVAL;
    } else if (bad_ptr(X) || ldx < m) {
        return CNMF_EINVAL;
    }
    if ((n + 255) / 256 > c->dev.num_cus || (m + 255) / 256 > c->dev.num_cus) return CNMF_EINVAL;
    const int p = prm->p;
    const int l = comp ? p + prm->nu : 0;
    const int T = prm->outer_iters;
    cnmf_trace tr{};
    if (trace) tr = *trace;

    Arena a;
    const size_t o_W = a.take<float>(32 * 32);
    const size_t o_BG = a.take<float>((size_t)n * p);
    const size_t o_BF = a.take<float>((size_t)m * p);
    const size_t o_FR = a.take<float>(32 * 32);
    const size_t o_GL = a.take<float>(32 * 32);
    const size_t o_L = a.take<double>(2);
    size_t part = std::max(sweep_right_partial_floats(c->dev, n, comp ? l : m),
                           sweep_left_partial_floats(c->dev, comp ? l : n, m));
    part = std::max(part, sweep_right_partial_floats(c->dev, p, m));       // F Q_R, F F^T
    part = std::max(part, sweep_left_partial_floats(c->dev, n, std::max(l, p)));  // Q_L^T G, G^T G
    part = std::max(part, sweep_right_partial_floats(c->dev, 32, 32));
    part = std::max(part, sweep_left_partial_floats(c->dev, 32, 32));
    const size_t o_part = a.take<float>(part);
    const size_t o_np = a.take<double>(nnls_partial_doubles(c->dev, std::max(n, m)));
    rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    const Dev& d = c->dev;
    float* W = at<float>(c, o_W);
    float* BG = at<float>(c, o_BG);
    float* BF = at<float>(c, o_BF);
    float* FR = at<float>(c, o_FR);
    float* GL = at<float>(c, o_GL);
    double* Ld = at<double>(c, o_L);
    float* pt = at<float>(c, o_part);
    double* np = at<double>(c, o_np);
    Control* ctl = c->ctl;

    // Subproblem data of Eq. (2) for the current F: W = F F^T, B = X F^T, or
    // Algorithm 1's F_R = F R, W = F_R F_R^T, B = X_R F_R^T.
    auto gdata = [&]() -> hipError_t {
        hipError_t e;
        if (comp) {
            if ((e = sweep_right(d, p, m, F, m, l, Q_R, l, false, FR, l, pt))) return e;
            if ((e = sweep_right(d, p, l, FR, l, p, FR, l, true, W, p, pt))) return e;
            return sweep_right(d, n, l, X_R, l, p, FR, l, true, BG, p, pt);
        }
        if ((e = sweep_right(d, p, m, F, m, p, F, m, true, W, p, pt))) return e;
        return sweep_right(d, n, m, X, ldx, p, F, m, true, BG, p, pt);
    };
    // Eq. (3) for the current G: W = G^T G, B^T = X^T G, or Algorithm 1's
    // G_L = L G, W = G_L^T G_L, B^T = X_L^T G_L.
    auto fdata = [&]() -> hipError_t {
        hipError_t e;
        if (comp) {
            if ((e = sweep_left(d, n, l, Q_L, l, p, G, p, GL, p, false, pt))) return e;
            if ((e = sweep_left(d, l, p, GL, p, p, GL, p, W, p, false, pt))) return e;
            return sweep_left(d, l, m, X_L, m, p, GL, p, BF, p, false, pt);
        }
        if ((e = sweep_left(d, n, p, G, p, p, G, p, W, p, false, pt))) return e;
        return sweep_left(d, n, m, X, ldx, p, G, p, BF, p, false, pt);
    };
    auto gargs = [&]() {
        NnlsArgs na{};
        na.rows = n; na.p = p; na.Z = G; na.z_rs = p; na.z_cs = 1; na.W = W; na.B = BG;
        na.L = Ld; na.inner_max = prm->inner_max; na.inner_min = prm->inner_min; na.forced = -1;
        return na;
    };
    auto fargs = [&]() {
        NnlsArgs na{};
        na.rows = m; na.p = p; na.Z = F; na.z_rs = 1; na.z_cs = m; na.W = W; na.B = BF;
        na.L = Ld; na.inner_max = prm->inner_max; na.inner_min = prm->inner_min; na.forced = -1;
        return na;
    };
    const bool global = prm->stop_rule == CNMF_STOP_GLOBAL;

    if (tr.ticks) CK(write_tick(d, (unsigned long long*)tr.ticks));
    if (T > 0 && global) {
        // Gradient bound: ratio * ||(P grad_G, P grad_F)|| at (G0, F0).
        CK(gdata());
        NnlsArgs na = gargs();
        na.pg_only = true;
        na.pg2_out = &ctl->pg2[0];
        CK(nnls(d, na, np, ctl));
        CK(fdata());
        na = fargs();
        na.pg_only = true;
        na.pg2_out = &ctl->pg2[1];
        CK(nnls(d, na, np, ctl));
        CK(tol_init(d, ctl, prm->inner_ratio));
    }
    if (tr.ticks && T > 0) CK(fill_u64(d, tr.ticks + 1, T, 0));
    for (int t = 0; t < T; ++t) {
        CK(gdata());
        CK(lipschitz(d, p, W, Ld, ctl));
        NnlsArgs na = gargs();
        if (global) { na.tol_ptr = &ctl->tol[0]; na.tol_state = &ctl->tol[0]; }
        else na.ratio = prm->inner_ratio;
        if (replay) na.forced_ptr = replay + 2 * t;
        if (tr.steps) na.steps_out = tr.steps + 2 * t;
        if (tr.lips) na.L_out = tr.lips + 2 * t;
        if (tr.tols) na.tol_out = tr.tols + 2 * t;
        if (tr.G_hist) na.hist = tr.G_hist + (size_t)t * n * p;
        CK(nnls(d, na, np, ctl));

        CK(fdata());
        CK(lipschitz(d, p, W, Ld + 1, ctl));
        na = fargs();
        na.L = Ld + 1;
        if (global) { na.tol_ptr = &ctl->tol[1]; na.tol_state = &ctl->tol[1]; }
        else na.ratio = prm->inner_ratio;
        if (replay) na.forced_ptr = replay + 2 * t + 1;
        if (tr.steps) na.steps_out = tr.steps + 2 * t + 1;
        if (tr.lips) na.L_out = tr.lips + 2 * t + 1;
        if (tr.tols) na.tol_out = tr.tols + 2 * t + 1;
        if (tr.F_hist) na.hist = tr.F_hist + (size_t)t * p * m;
        if (tr.ticks) na.tick_out = (unsigned long long*)(tr.ticks + 1 + t);
        CK(nnls(d, na, np, ctl));
    }
    return CNMF_OK;
}

int cnmf_rre(cnmf_ctx* c, int64_t n, int64_t m, const float* X, int64_t ldx, int32_t p,
             const float* G, int64_t strideG, const float* F, int64_t strideF, int32_t count,
             double* out) {
    if (!c || n < 1 || m < 1 || p < 1 || p > 32 || count < 0) return CNMF_EINVAL;
    if (count == 0) return CNMF_OK;
    if (bad_ptr(X) || bad_ptr(G) || bad_ptr(F) || bad_ptr(out) || ldx < m) return CNMF_EINVAL;
    Arena a;
    const size_t len = rre_partial_doubles(c->dev, n, m, count);
    const size_t off = a.take<double>(len);
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    return from_hip(rre(c->dev, n, m, X, ldx, p, G, strideG, F, strideF, count, out,
                        at<double>(c, off), (int64_t)len));
}

}  // extern "C"
