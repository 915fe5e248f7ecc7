// C ABI of libcnmf: argument validation, workspace, and the enqueue order of
// randomized subspace iteration (Sec. 3, Algorithm 2) and of the plain and
// compressed NeNMF outer loops (Sec. 2; Sec. 3, Algorithm 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "ctx.hpp"

namespace {
int scratch_address(int device, char** out);   // below, beside the scratch it serves
}

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
        case CNMF_ENODERIV: return "no derivative: the rank rule replaced a basis column";
        case CNMF_ETOOBIG: return "the problem needs more than the no-alloc scratch holds";
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
    if (hipMalloc((void**)&c->slots, kSlotWords * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void**)&c->oxch, orth_exchange_words() * sizeof(uint64_t)) != hipSuccess) {
        (void)hipFree(c->ctl);
        if (c->slots) (void)hipFree(c->slots);
        delete c;
        return CNMF_ENOMEM;
    }
    if (hipMemset(c->ctl, 0, sizeof(Control)) != hipSuccess ||
        hipMemset(c->slots, 0, kSlotWords * sizeof(uint64_t)) != hipSuccess ||
        hipMemset(c->oxch, 0, orth_exchange_words() * sizeof(uint64_t)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->ctl);
        (void)hipFree(c->slots);
        (void)hipFree(c->oxch);
        delete c;
        return CNMF_EHIP;
    }
    {
        float* host = new (std::nothrow) float[kBetaLen];
        bool good = host != nullptr && hipMalloc((void**)&c->beta, kBetaLen * sizeof(float)) == hipSuccess;
        if (good) {
            momentum_table(host, kBetaLen);
            good = hipMemcpy(c->beta, host, kBetaLen * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
        }
        delete[] host;
        if (!good) {
            (void)hipFree(c->ctl);
            (void)hipFree(c->slots);
            (void)hipFree(c->oxch);
            if (c->beta) (void)hipFree(c->beta);
            delete c;
            return CNMF_ENOMEM;
        }
    }
    {   // the device's copy of the no-alloc scratch (device current)
        const int src = scratch_address(device, &c->scratch);
        if (src) {
            (void)hipFree(c->ctl);
            (void)hipFree(c->slots);
            (void)hipFree(c->oxch);
            (void)hipFree(c->beta);
            delete c;
            return src;
        }
    }
    if (const char* e = std::getenv("CNMF_DLAG")) {
        const int v = std::atoi(e);
        if ((v >= 0 && v <= 4) || v == kGrouped) c->dlag = v;
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
    if (c->slots) (void)hipFree(c->slots);
    if (c->oxch) (void)hipFree(c->oxch);
    if (c->beta) (void)hipFree(c->beta);
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

int cnmf_sweep_dual(cnmf_ctx* c, int64_t R, int64_t C, const float* X, int64_t ldx, int32_t k,
                    const float* AT, int64_t ldat, const float* B, int64_t ldb, float* Y,
                    int64_t ldy, float* Z, int64_t ldz, int32_t z_trans) {
    if (!c || R < 1 || C < 1 || k < 1 || k > 32) return CNMF_EINVAL;
    if (bad_ptr(X) || bad_ptr(AT) || bad_ptr(B) || bad_ptr(Y) || bad_ptr(Z)) return CNMF_EINVAL;
    if (ldx < C || ldat < C || ldb < k || ldy < k || (z_trans ? ldz < C : ldz < k))
        return CNMF_EINVAL;
    Arena a;
    size_t off = a.take<float>(sweep_dual_partial_floats(c->dev, R, C));
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    return from_hip(sweep_dual(c->dev, R, C, X, ldx, k, AT, ldat, B, ldb, Y, ldy, Z, ldz,
                               z_trans != 0, at<float>(c, off)));
}

int cnmf_sweep_dual_bf16(cnmf_ctx* c, int64_t R, int64_t C, const uint16_t* Xb, int64_t ldxb,
                         int32_t k, const float* AT, int64_t ldat, const float* B, int64_t ldb,
                         float* Y, int64_t ldy, float* Z, int64_t ldz, int32_t z_trans) {
    if (!c || R < 1 || C < 1 || k < 1 || k > 32) return CNMF_EINVAL;
    if (bad_ptr(Xb) || bad_ptr(AT) || bad_ptr(B) || bad_ptr(Y) || bad_ptr(Z)) return CNMF_EINVAL;
    if (ldxb < C || ldat < C || ldb < k || ldy < k || (z_trans ? ldz < C : ldz < k))
        return CNMF_EINVAL;
    Arena a;
    size_t off = a.take<float>(sweep_dual_bf16_partial_floats(c->dev, R, C));
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    return from_hip(sweep_dual_bf16(c->dev, R, C, Xb, ldxb, k, AT, ldat, B, ldb, Y, ldy, Z, ldz,
                                    z_trans != 0, at<float>(c, off)));
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

int cnmf_sweep_right_bf16(cnmf_ctx* c, int64_t R, int64_t C, const uint16_t* Xb, int64_t ldxb,
                          int32_t k, const float* A, int64_t lda, int32_t a_trans, float* Y,
                          int64_t ldy) {
    if (!c || R < 1 || C < 1 || k < 1 || k > 32) return CNMF_EINVAL;
    if (bad_ptr(Xb) || bad_ptr(A) || bad_ptr(Y) || ldxb < C || ldy < k) return CNMF_EINVAL;
    if (a_trans ? lda < C : lda < k) return CNMF_EINVAL;
    Arena a;
    const size_t off = a.take<float>(sweep_right_bf16_partial_floats(c->dev, R, C));
    const size_t opk = a.take<uint16_t>(bf16_pack_elems(C));
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    return from_hip(sweep_right_bf16(c->dev, R, C, Xb, ldxb, k, A, lda, a_trans != 0, Y, ldy,
                                     at<float>(c, off), at<uint16_t>(c, opk)));
}

int cnmf_sweep_left_bf16(cnmf_ctx* c, int64_t R, int64_t C, const uint16_t* Xb, int64_t ldxb,
                         int32_t k, const float* B, int64_t ldb, float* Z, int64_t ldz,
                         int32_t z_trans) {
    if (!c || R < 1 || C < 1 || k < 1 || k > 32) return CNMF_EINVAL;
    if (bad_ptr(Xb) || bad_ptr(B) || bad_ptr(Z) || ldxb < C || ldb < k) return CNMF_EINVAL;
    if (z_trans ? ldz < C : ldz < k) return CNMF_EINVAL;
    Arena a;
    const size_t off = a.take<float>(sweep_left_bf16_partial_floats(c->dev, R, C));
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    return from_hip(sweep_left_bf16(c->dev, R, C, Xb, ldxb, k, B, ldb, Z, ldz, z_trans != 0,
                                    at<float>(c, off)));
}

int cnmf_orth(cnmf_ctx* c, int64_t N, int32_t l, const float* Y, const float* pool,
              int32_t pool_trans, double tau2, float* Q, int32_t* replaced) {
    if (!c || N < 1 || l < 1 || l > 32 || l > N) return CNMF_EINVAL;
    if (bad_ptr(Y) || bad_ptr(pool) || bad_ptr(Q)) return CNMF_EINVAL;
    if (!(tau2 > 0.0 && tau2 < 1.0)) return CNMF_EINVAL;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    unsigned seq = 0;
    CK(next_seq(c, &seq));
    return from_hip(orth(c->dev, N, l, Y, pool, pool_trans != 0, tau2, Q, nullptr, 0, replaced,
                         c->oxch, seq, c->ctl));
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
    int tiles = 0;
    unsigned nblk = 0;
    if (rows > CNMF_MAX_ROWS || !phase_grid(c->dev, rows, &tiles, &nblk)) return CNMF_EINVAL;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    PhaseArgs a{};
    a.rows = rows;
    a.p = p;
    a.mode = 0;
    a.Z = Z;
    a.z_rs = z_rs;
    a.z_cs = z_cs;
    a.Wgiven = W;
    a.Bgiven = B;
    a.slot_s = c->slots;
    a.slot_pg = c->slots + 1024;
    a.beta = c->beta;
    a.ctl = c->ctl;
    a.tol_value = tol;
    a.inner_max = inner_max;
    a.inner_min = inner_min;
    a.forced = forced;
    a.dlag = c->dlag;
    a.steps_out = steps_out;
    a.L_out = L_out;
    a.pg2_out = pg2_out;
    CK(next_seq(c, &a.seq));
    return from_hip(phase(c->dev, a, nblk, tiles));
}

// ---------------------------------------------------------------------------
// Randomized subspace iteration (Algorithm 2)
// ---------------------------------------------------------------------------

}  // extern "C"

int rsi_run(cnmf_ctx* c, int64_t n, int64_t m, const float* X, const uint16_t* Xb,
                    int64_t ldx, const cnmf_params* prm, const float* oL, const float* oR,
                    float* QL_out, float* QR_out, float* XL_out, float* XR_out) {
    const int l = prm->p + prm->nu;
    const bool bf = Xb != nullptr;
    const int64_t ldt = (m + 3) / 4 * 4;       // pitch of the transposed m-space panels
    Arena a;
    const size_t o_oRt = a.take<float>((size_t)n * l);
    const size_t o_Yn = a.take<float>((size_t)n * l);
    const size_t o_QL = a.take<float>((size_t)n * l);
    const size_t o_Ym = a.take<float>((size_t)m * l);
    const size_t o_QRt = a.take<float>((size_t)m * l);
    const size_t o_oLT = a.take<float>((size_t)l * ldt);
    const size_t o_QRtT = a.take<float>((size_t)l * ldt);
    const size_t o_QLtT = a.take<float>((size_t)l * ldt);
    const size_t part = bf ? sweep_dual_bf16_partial_floats(c->dev, n, m)
                           : sweep_dual_partial_floats(c->dev, n, m);
    const size_t o_part = a.take<float>(part);
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    const Dev& d = c->dev;
    float* oRt = at<float>(c, o_oRt);
    float* Yn = at<float>(c, o_Yn);
    float* QL = at<float>(c, o_QL);
    float* Ym = at<float>(c, o_Ym);
    float* QRt = at<float>(c, o_QRt);
    float* oLT = at<float>(c, o_oLT);
    float* QRtT = at<float>(c, o_QRtT);
    float* QLtT = at<float>(c, o_QLtT);
    float* pt = at<float>(c, o_part);
    const double tau2 = prm->tau2;

    // Y (n x l) = X A with A (m x l) given as its transpose AT (l x ldt) and
    // Z = X^T B, one product for each chain, in one read of X (BF16 form:
    // X in bfloat16, the skinny operands rounded to bfloat16)
    auto both = [&](const float* AT, float* Y, const float* B, float* Z, bool trans) -> hipError_t {
        if (bf)
            return sweep_dual_bf16(d, n, m, Xb, ldx, l, AT, ldt, B, l, Y, l, Z, trans ? m : l,
                                   trans, pt);
        return sweep_dual(d, n, m, X, ldx, l, AT, ldt, B, l, Y, l, Z, trans ? m : l, trans, pt);
    };
    // orthonormal bases of an n-space panel Yn_ (n x l, pool Omega_R^T) and an
    // m-space panel Ym_ (m x l, pool Omega_L) at once (independent panels);
    // QmT: optional transposed copy (l x ldt)
    uint64_t* xch2 = c->oxch + orth_exchange_words() / 2;
    auto orth_nm = [&](const float* Yn_, float* Qn, const float* Ym_, float* Qm,
                       float* QmT) -> hipError_t {
        unsigned sa = 0, sb = 0;
        hipError_t e = next_seq(c, &sa);
        if (e == hipSuccess) e = next_seq(c, &sb);
        if (e != hipSuccess) return e;
        const OrthArgs ga = orth_args(n, l, Yn_, oRt, false, tau2, Qn, nullptr, 0, nullptr, c->oxch,
                                      sa, c->ctl, orth_pair_blocks(d, n));
        const OrthArgs gb = orth_args(m, l, Ym_, oL, false, tau2, Qm, QmT, ldt, nullptr, xch2, sb,
                                      c->ctl, orth_pair_blocks(d, m));
        return orth_pair(d, ga, gb);
    };

    if (!bf && (prm->flags & CNMF_FLAG_VALIDATE_INPUT)) CK(check_input(d, n, m, X, ldx, c->ctl));
    CK(transpose(d, l, n, oR, n, oRt, l));                       // Omega_R^T, n x l
    CK(transpose(d, m, l, oL, l, oLT, ldt));                     // Omega_L^T, l x m
    // The two chains (left and right bases) are independent: each pair of
    // bases that both chains need at the same point is found in one launch.
    // Step 0: sketches X Omega_L and (Omega_R X)^T and their bases.
    CK(both(oLT, Yn, oRt, Ym, false));
    CK(orth_nm(Yn, QL, Ym, QRt, QRtT));
    for (int k = 1; k <= prm->q; ++k) {
        // Q~_L^(k) = orth(X^T Q_L^(k-1)), kept in the Q_R output (m x l), and
        // Q~_R^(k)^T = orth(X Q_R^(k-1)^T), kept in the Q_L output (n x l).
        CK(both(QRtT, Yn, QL, Ym, false));
        CK(orth_nm(Yn, QL_out, Ym, QR_out, QLtT));
        // X Q~_L^(k) (n x l) and (Q~_R^(k) X)^T (m x l).
        if (k < prm->q) {
            CK(both(QLtT, XR_out, QL_out, Ym, false));
            CK(orth_nm(XR_out, QL, Ym, QRt, QRtT));
        } else {
            CK(both(QLtT, XR_out, QL_out, XL_out, true));   // X_L = Q_L^T X, l x m
        }
    }
    return CNMF_OK;
}

extern "C" {

int cnmf_rsi(cnmf_ctx* c, int64_t n, int64_t m, const float* X, int64_t ldx,
             const cnmf_params* prm, const float* omega_L, const float* omega_R, float* Q_L,
             float* Q_R, float* X_L, float* X_R) {
    if (!c || n < 1 || m < 1) return CNMF_EINVAL;
    int rc = check_params(prm, n, m, true);
    if (rc) return rc;
    if (prm->sweep_prec != CNMF_PREC_FP32) return CNMF_EINVAL;
    if (bad_ptr(X) || ldx < m || bad_ptr(omega_L) || bad_ptr(omega_R)) return CNMF_EINVAL;
    if (bad_ptr(Q_L) || bad_ptr(Q_R) || bad_ptr(X_L) || bad_ptr(X_R)) return CNMF_EINVAL;
    return rsi_run(c, n, m, X, nullptr, ldx, prm, omega_L, omega_R, Q_L, Q_R, X_L, X_R);
}

int cnmf_rsi_bf16(cnmf_ctx* c, int64_t n, int64_t m, const uint16_t* Xb, int64_t ldxb,
                  const cnmf_params* prm, const float* omega_L, const float* omega_R,
                  float* Q_L, float* Q_R, float* X_L, float* X_R) {
    if (!c || n < 1 || m < 1) return CNMF_EINVAL;
    int rc = check_params(prm, n, m, true);
    if (rc) return rc;
    if (bad_ptr(Xb) || ldxb < m) return CNMF_EINVAL;
    if (bad_ptr(omega_L) || bad_ptr(omega_R)) return CNMF_EINVAL;
    if (bad_ptr(Q_L) || bad_ptr(Q_R) || bad_ptr(X_L) || bad_ptr(X_R)) return CNMF_EINVAL;
    return rsi_run(c, n, m, nullptr, Xb, ldxb, prm, omega_L, omega_R, Q_L, Q_R, X_L, X_R);
}

}  // extern "C"

namespace {

// The two variants of the compression of Sec. 3 that Algorithm 2 improves
// on: the scaled Gaussian projection and power iteration without
// re-orthonormalisation (the same chains as rsi_run, orthonormalised once).
int compress_variant(cnmf_ctx* c, int kind, int64_t n, int64_t m, const float* X, int64_t ldx,
                     const cnmf_params* prm, const float* oL, const float* oR, float* QL_out,
                     float* QR_out, float* XL_out, float* XR_out) {
    const int l = prm->p + prm->nu;
    const int64_t ldt = (m + 3) / 4 * 4;
    const bool power = kind == CNMF_COMPRESS_POWER;
    Arena a;
    const size_t o_YmT = a.take<float>((size_t)l * ldt);
    const size_t o_YmTb = a.take<float>(power ? (size_t)l * ldt : 1);
    const size_t o_QRT = a.take<float>(power ? (size_t)l * ldt : 1);
    const size_t o_YnA = a.take<float>(power ? (size_t)n * l : 1);
    const size_t o_YnB = a.take<float>(power ? (size_t)n * l : 1);
    const size_t o_Ym = a.take<float>(power ? (size_t)m * l : 1);
    const size_t o_oRt = a.take<float>(power ? (size_t)n * l : 1);
    const size_t o_nrm = a.take<double>(kNormBlocks);
    const size_t o_part = a.take<float>(std::max(sweep_right_partial_floats(c->dev, n, m),
                                                 sweep_left_partial_floats(c->dev, n, m)));
    int rc = ensure_ws(c, a.off);
    if (rc) return rc;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    const Dev& d = c->dev;
    float* YmT = at<float>(c, o_YmT);
    float* pt = at<float>(c, o_part);
    double* nrm = at<double>(c, o_nrm);
    auto right = [&](const float* AT, float* Y) {      // Y (n x l) = X A, A given as l x ldt
        return sweep_right(d, n, m, X, ldx, l, AT, ldt, true, Y, l, pt);
    };
    // Z = X^T B, written m x l (ldz = l) or transposed l x m with pitch ldz
    auto left = [&](const float* B, float* Z, bool trans, int64_t ldz) {
        return sweep_left(d, n, m, X, ldx, l, B, l, Z, ldz, trans, pt);
    };
    if (prm->flags & CNMF_FLAG_VALIDATE_INPUT) CK(check_input(d, n, m, X, ldx, c->ctl));
    if (!power) {
        // L = Omega_R / sqrt(l) (l x n), R = Omega_L / sqrt(l) (m x l)
        const float s = (float)(1.0 / std::sqrt((double)l));
        CK(transpose(d, m, l, oL, l, YmT, ldt));                 // Omega_L^T
        CK(scale2d(d, l, m, YmT, ldt, YmT, ldt, s));             // R^T
        CK(scale2d(d, m, l, oL, l, QR_out, l, s));               // Q_R = R
        CK(transpose(d, l, n, oR, n, QL_out, l));                // Omega_R^T
        CK(scale2d(d, n, l, QL_out, l, QL_out, l, s));           // Q_L = L^T
        CK(right(YmT, XR_out));                                  // X_R = X R
        CK(left(QL_out, XL_out, true, m));                       // X_L = L X (l x m)
        return CNMF_OK;
    }
    float* YmTb = at<float>(c, o_YmTb);
    float* QRT = at<float>(c, o_QRT);
    float* YnA = at<float>(c, o_YnA);
    float* YnB = at<float>(c, o_YnB);
    float* Ym = at<float>(c, o_Ym);
    float* oRt = at<float>(c, o_oRt);
    CK(transpose(d, m, l, oL, l, YmT, ldt));                     // Omega_L^T
    CK(transpose(d, l, n, oR, n, oRt, l));                       // Omega_R^T
    // chain A: (X^T X)^q Omega_L, kept transposed between products;
    // chain B: (X X^T)^q Omega_R^T.  Each product is scaled to unit
    // Frobenius norm (its range is unchanged).
    for (int k = 1; k <= prm->q; ++k) {
        CK(right(YmT, YnA));
        CK(normalize2d(d, n, l, YnA, l, nrm));
        if (k < prm->q) {
            CK(left(YnA, YmT, true, ldt));
            CK(normalize2d(d, l, m, YmT, ldt, nrm));
        } else {
            CK(left(YnA, Ym, false, l));
            CK(normalize2d(d, m, l, Ym, l, nrm));
        }
        CK(left(k == 1 ? oRt : YnB, YmTb, true, ldt));
        CK(normalize2d(d, l, m, YmTb, ldt, nrm));
        CK(right(YmTb, YnB));
        CK(normalize2d(d, n, l, YnB, l, nrm));
    }
    unsigned sa = 0, sb = 0;
    CK(next_seq(c, &sa));
    CK(next_seq(c, &sb));
    const OrthArgs ga = orth_args(n, l, YnB, oRt, false, prm->tau2, QL_out, nullptr, 0, nullptr,
                                  c->oxch, sa, c->ctl, orth_pair_blocks(d, n));
    const OrthArgs gb = orth_args(m, l, Ym, oL, false, prm->tau2, QR_out, QRT, ldt, nullptr,
                                  c->oxch + orth_exchange_words() / 2, sb, c->ctl,
                                  orth_pair_blocks(d, m));
    CK(orth_pair(d, ga, gb));
    CK(right(QRT, XR_out));                                      // X_R = X Q_R
    CK(left(QL_out, XL_out, true, m));                           // X_L = Q_L^T X
    return CNMF_OK;
}

}  // namespace

extern "C" {

int cnmf_compress(cnmf_ctx* c, int32_t kind, int64_t n, int64_t m, const float* X, int64_t ldx,
                  const cnmf_params* prm, const float* omega_L, const float* omega_R, float* Q_L,
                  float* Q_R, float* X_L, float* X_R) {
    if (!c || n < 1 || m < 1) return CNMF_EINVAL;
    if (kind != CNMF_COMPRESS_RSI && kind != CNMF_COMPRESS_GAUSSIAN && kind != CNMF_COMPRESS_POWER)
        return CNMF_EINVAL;
    int rc = check_params(prm, n, m, true);
    if (rc) return rc;
    if (prm->sweep_prec != CNMF_PREC_FP32) return CNMF_EINVAL;
    if (bad_ptr(X) || ldx < m || bad_ptr(omega_L) || bad_ptr(omega_R)) return CNMF_EINVAL;
    if (bad_ptr(Q_L) || bad_ptr(Q_R) || bad_ptr(X_L) || bad_ptr(X_R)) return CNMF_EINVAL;
    if (kind == CNMF_COMPRESS_RSI)
        return rsi_run(c, n, m, X, nullptr, ldx, prm, omega_L, omega_R, Q_L, Q_R, X_L, X_R);
    return compress_variant(c, kind, n, m, X, ldx, prm, omega_L, omega_R, Q_L, Q_R, X_L, X_R);
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

}  // extern "C"

// Scratch of cnmf_solve_noalloc: device memory of the library itself, one
// copy per GPU (each device holds it from the load of the library until the
// process ends).  Host code never passes `scratch` itself to a kernel (in
// host code the name is only a stand-in for the device symbol): every use
// goes through the address hipGetSymbolAddress returned for the device,
// kept in g_scratch by scratch_address().
static __device__ __align__(256) char scratch[CNMF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `device` (current), looked up once per
// device.
int scratch_address(int device, char** out) {
    if (device < 0 || device >= kMaxDevices) return CNMF_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return CNMF_EHIP;
        g_scratch[device] = static_cast<char*>(ptr);
    }
    *out = g_scratch[device];
    return CNMF_OK;
}

// The outer loop of cnmf_solve.  ws: workspace base of at least `cap`
// bytes, or null for the context's (growing) workspace.
// CNMF_FUSED_LOOP=0 runs the compressed outer loop as one launch per phase
// (the form every other configuration uses), for comparison.
bool fused_loop_enabled() {
    static const bool on = [] {
        const char* e = std::getenv("CNMF_FUSED_LOOP");
        return !(e && e[0] == '0');
    }();
    return on;
}

int solve_run(cnmf_ctx* c, char* ws, size_t cap, int method, int64_t n, int64_t m,
              const float* X, int64_t ldx, const float* Q_L, const float* Q_R,
              const float* X_L, const float* X_R, const cnmf_params* prm, float* G, float* F,
              const cnmf_trace* trace, const int32_t* replay) {
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
    int tilesG = 0, tilesF = 0;
    unsigned nbG = 0, nbF = 0;
    if (n > CNMF_MAX_ROWS || m > CNMF_MAX_ROWS) return CNMF_EINVAL;
    if (!phase_grid(c->dev, n, &tilesG, &nbG) || !phase_grid(c->dev, m, &tilesF, &nbF))
        return CNMF_EINVAL;
    const int p = prm->p;
    const int l = comp ? p + prm->nu : 0;
    const int T = prm->outer_iters;
    cnmf_trace tr{};
    if (trace) tr = *trace;

    Arena ar;
    const size_t o_pG = ar.take<float>((size_t)nbG * 1024);
    const size_t o_pF = ar.take<float>((size_t)nbF * 1024);
    const size_t o_BG = ar.take<float>(comp ? 1 : (size_t)n * p);
    const size_t o_BF = ar.take<float>(comp ? 1 : (size_t)m * p);
    const size_t o_sw = ar.take<float>(comp ? 1 : std::max(sweep_right_partial_floats(c->dev, n, m),
                                                            sweep_left_partial_floats(c->dev, n, m)));
    const size_t o_eig = ar.take<double>(4 * kEigWords);   // {L, v} per side and parity
    // the whole outer loop in one launch: compressed Nesterov, the default
    // stop-test lag, row tiles the fused kernel covers
    const bool budget = prm->time_budget > 0.0;
    const bool fused = comp && T > 0 && prm->solver == CNMF_SOLVER_NESTEROV &&
                       prm->restart == CNMF_RESTART_NONE && c->dlag < 0 &&
                       fused_loop_enabled() && phase_loop_supported(p, tilesG, tilesF);
    const size_t o_pG64 = ar.take<uint64_t>(fused ? (size_t)nbG * 1024 : 1);
    const size_t o_pF64 = ar.take<uint64_t>(fused ? (size_t)nbF * 1024 : 1);
    const size_t o_largs = ar.take<LoopArgs>(1);
    const size_t o_stopw = ar.take<uint64_t>(1);
    if (ws) {
        if (ar.off > cap) return CNMF_ETOOBIG;
    } else {
        rc = ensure_ws(c, ar.off);
        if (rc) return rc;
        ws = c->ws;
    }
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    const Dev& d = c->dev;
    float* pG = reinterpret_cast<float*>(ws + o_pG);
    float* pF = reinterpret_cast<float*>(ws + o_pF);
    float* BG = reinterpret_cast<float*>(ws + o_BG);
    float* BF = reinterpret_cast<float*>(ws + o_BF);
    float* sw = reinterpret_cast<float*>(ws + o_sw);
    double* eig = reinterpret_cast<double*>(ws + o_eig);
    uint64_t* pG64 = reinterpret_cast<uint64_t*>(ws + o_pG64);
    uint64_t* pF64 = reinterpret_cast<uint64_t*>(ws + o_pF64);
    auto eig_at = [&](int side, int par) { return eig + (size_t)(2 * side + par) * kEigWords; };
    Control* ctl = c->ctl;
    const bool global = prm->stop_rule == CNMF_STOP_GLOBAL;

    PhaseArgs base{};
    base.p = p;
    base.ell = l;
    base.mode = comp ? 2 : 1;
    base.slot_s = c->slots;
    base.slot_pg = c->slots + 1024;
    base.beta = c->beta;
    base.ctl = ctl;
    base.inner_max = prm->inner_max;
    base.inner_min = prm->inner_min;
    base.forced = -1;
    base.dlag = c->dlag;
    base.solver = prm->solver == CNMF_SOLVER_HALS ? kSolverHals
                : prm->solver == CNMF_SOLVER_MU   ? kSolverMu
                : prm->restart == CNMF_RESTART_GRADIENT ? kSolverRestart
                                                        : kSolverNesterov;
    // G update (Eq. (2) / Algorithm 1 with X_R, F_R): rows of G
    PhaseArgs ga = base;
    ga.rows = n;
    ga.Z = G;
    ga.z_rs = p;
    ga.z_cs = 1;
    ga.wt = 0;
    ga.D = X_R;
    ga.d_rs = l;
    ga.d_cs = 1;
    ga.Q = Q_L;
    ga.Bgiven = BG;
    ga.part_in = pF;
    ga.nin = (int)nbF;
    ga.part_out = pG;
    // F update (Eq. (3) / Algorithm 1 with X_L, G_L): columns of F
    PhaseArgs fa = base;
    fa.rows = m;
    fa.Z = F;
    fa.z_rs = 1;
    fa.z_cs = m;
    fa.wt = 1;
    fa.D = X_L;
    fa.d_rs = 1;
    fa.d_cs = m;
    fa.Q = Q_R;
    fa.Bgiven = BF;
    fa.part_in = pG;
    fa.nin = (int)nbG;
    fa.part_out = pF;

    unsigned last_seq = 0;
    auto run = [&](PhaseArgs a, bool is_g) -> hipError_t {
        hipError_t e = next_seq(c, &a.seq);
        if (e != hipSuccess) return e;
        last_seq = a.seq;
        return phase(d, a, is_g ? nbG : nbF, is_g ? tilesG : tilesF);
    };
    auto bg = [&]() -> hipError_t {   // plain: B_G = X F^T
        return comp ? hipSuccess : sweep_right(d, n, m, X, ldx, p, F, m, true, BG, p, sw);
    };
    auto bf = [&]() -> hipError_t {   // plain: B_F^T = X^T G
        return comp ? hipSuccess : sweep_left(d, n, m, X, ldx, p, G, p, BF, p, false, sw);
    };

    if (tr.ticks) CK(write_tick(d, (unsigned long long*)tr.ticks));
    if (fused) {
        // tagged partials: tag 0 is never issued, so cleared words read as absent
        CK(fill_u64(d, pG64, (int64_t)nbG * 1024, 0));
        CK(fill_u64(d, pF64, (int64_t)nbF * 1024, 0));
        CK(fill_u64(d, reinterpret_cast<uint64_t*>(ws + o_stopw), 1, 0));
        ga.part_in = nullptr;
        ga.part_out = nullptr;
        ga.part_in64 = pF64;
        ga.part_out64 = pG64;
        fa.part_in = nullptr;
        fa.part_out = nullptr;
        fa.part_in64 = pG64;
        fa.part_out64 = pF64;
    }
    if (budget) {
        const double ticks = prm->time_budget * c->clock_hz;
        CK(arm_deadline(d, ctl, ticks < 1.8e19 ? (unsigned long long)ticks : ~0ull >> 1));
    }
    if (tr.outer_done) CK(fill_i32(d, tr.outer_done, 1, 0));
    {   // partial product of F0 for the first G update
        PhaseArgs a = fa;
        a.kind = 2;
        CK(run(a, false));
    }
    unsigned seq_pF = last_seq;   // tag of the partials now in pF64 (fused)
    if (T > 0 && global) {
        // gradient bound: ratio * ||(P grad_G, P grad_F)|| at (G0, F0)
        CK(bg());
        PhaseArgs a = ga;
        a.kind = 1;
        a.pg2_out = &ctl->pg2[0];
        a.seq_in = seq_pF;
        CK(run(a, true));
        const unsigned seq_pG = last_seq;
        CK(bf());
        a = fa;
        a.kind = 1;
        a.pg2_out = &ctl->pg2[1];
        a.tol_init_from = &ctl->pg2[0];
        a.tol_init_out = &ctl->tol[0];
        a.ratio = prm->inner_ratio;
        a.seq_in = seq_pG;
        CK(run(a, false));
        seq_pF = last_seq;
    }
    if (fused) {
        if (tr.ticks) CK(fill_u64(d, tr.ticks + 1, T, 0));
        LoopArgs L{};
        L.g = ga;
        L.f = fa;
        if (global) {
            L.g.tol_state = &ctl->tol[0];   // marks the global rule; the loop keeps the bounds itself
            L.f.tol_state = &ctl->tol[1];
        } else {
            L.g.ratio = prm->inner_ratio;
            L.f.ratio = prm->inner_ratio;
        }
        if (replay) {
            L.g.forced_ptr = replay;
            L.f.forced_ptr = replay + 1;
        }
        if (tr.steps) { L.g.steps_out = tr.steps; L.f.steps_out = tr.steps + 1; }
        if (tr.lips) { L.g.L_out = tr.lips; L.f.L_out = tr.lips + 1; }
        if (tr.tols) { L.g.tol_out = tr.tols; L.f.tol_out = tr.tols + 1; }
        L.g.hist = tr.G_hist;
        L.f.hist = tr.F_hist;
        if (tr.W_hist) { L.g.w_out = tr.W_hist; L.f.w_out = tr.W_hist + (size_t)p * p; }
        if (tr.ticks) L.f.tick_out = (unsigned long long*)(tr.ticks + 1);
        L.f.done_out = tr.outer_done;
        if (budget) {   // block 0 publishes its verdict after every F phase
            L.f.deadline = &ctl->deadline;
            L.f.stop_word = reinterpret_cast<uint64_t*>(ws + o_stopw);
        }
        L.T = T;
        L.nbG = nbG;
        L.nbF = nbF;
        L.seq_pre = seq_pF;
        CK(reserve_seq(c, 2u * (unsigned)T, &L.seq0));
        L.g_hist_stride = (int64_t)n * p;
        L.f_hist_stride = (int64_t)p * m;
        L.global_rule = global ? 1 : 0;
        CK(phase_loop(d, L, reinterpret_cast<LoopArgs*>(ws + o_largs), tilesG, tilesF));
        return CNMF_OK;
    }
    if (tr.ticks && T > 0) CK(fill_u64(d, tr.ticks + 1, T, 0));
    // no warm start for the first subproblem of either side
    CK(fill_u64(d, reinterpret_cast<uint64_t*>(eig), 4 * kEigWords, 0));
    for (int t = 0; t < T; ++t) {
        CK(bg());
        PhaseArgs a = ga;
        if (global) { a.tol_ptr = &ctl->tol[0]; a.tol_state = &ctl->tol[0]; }
        else a.ratio = prm->inner_ratio;
        if (replay) a.forced_ptr = replay + 2 * t;
        if (tr.steps) a.steps_out = tr.steps + 2 * t;
        if (tr.lips) a.L_out = tr.lips + 2 * t;
        if (tr.tols) a.tol_out = tr.tols + 2 * t;
        if (tr.G_hist) a.hist = tr.G_hist + (size_t)t * n * p;
        a.eig_in = eig_at(0, (t + 1) & 1);
        a.eig_out = eig_at(0, t & 1);
        if (tr.W_hist) a.w_out = tr.W_hist + (size_t)(2 * t) * p * p;
        if (budget) a.stop_flag = &ctl->stop;
        CK(run(a, true));
        CK(bf());
        a = fa;
        if (global) { a.tol_ptr = &ctl->tol[1]; a.tol_state = &ctl->tol[1]; }
        else a.ratio = prm->inner_ratio;
        if (replay) a.forced_ptr = replay + 2 * t + 1;
        if (tr.steps) a.steps_out = tr.steps + 2 * t + 1;
        if (tr.lips) a.L_out = tr.lips + 2 * t + 1;
        if (tr.tols) a.tol_out = tr.tols + 2 * t + 1;
        if (tr.F_hist) a.hist = tr.F_hist + (size_t)t * p * m;
        if (tr.ticks) a.tick_out = (unsigned long long*)(tr.ticks + 1 + t);
        a.eig_in = eig_at(1, (t + 1) & 1);
        a.eig_out = eig_at(1, t & 1);
        if (tr.W_hist) a.w_out = tr.W_hist + (size_t)(2 * t + 1) * p * p;
        if (tr.outer_done) {
            a.done_out = tr.outer_done;
            a.done_value = t + 1;
        }
        if (budget) {
            a.stop_flag = &ctl->stop;
            a.deadline = &ctl->deadline;
        }
        CK(run(a, false));
    }
    return CNMF_OK;
}

}  // namespace

extern "C" {

int cnmf_solve(cnmf_ctx* c, int method, int64_t n, int64_t m, const float* X, int64_t ldx,
               const float* Q_L, const float* Q_R, const float* X_L, const float* X_R,
               const cnmf_params* prm, float* G, float* F, const cnmf_trace* trace,
               const int32_t* replay) {
    return solve_run(c, nullptr, 0, method, n, m, X, ldx, Q_L, Q_R, X_L, X_R, prm, G, F, trace,
                     replay);
}

int cnmf_solve_noalloc(cnmf_ctx* c, int method, int64_t n, int64_t m, const float* X,
                       int64_t ldx, const float* Q_L, const float* Q_R, const float* X_L,
                       const float* X_R, const cnmf_params* prm, float* G, float* F,
                       const cnmf_trace* trace, const int32_t* replay) {
    if (!c || !c->scratch) return CNMF_EINVAL;
    return solve_run(c, c->scratch, CNMF_NOALLOC_SCRATCH_BYTES, method, n, m, X, ldx, Q_L, Q_R,
                     X_L, X_R, prm, G, F, trace, replay);
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
