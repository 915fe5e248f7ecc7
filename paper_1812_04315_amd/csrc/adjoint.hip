// Differentiation form: reverse mode of compressed NeNMF (Sec. 3,
// Algorithms 1 and 2) unrolled over T outer iterations with exactly K inner
// Nesterov steps each (Sec. 2), giving dL/dX for a loss L(G_T, F_T).
//
// Forward: randomized subspace iteration keeping every sketch panel and its
// basis (the tape), then the outer loop on the single-instance solver,
// keeping (G, F) every `ckpt` outer iterations.  Backward: each segment of
// `ckpt` iterations is recomputed from its checkpoint; every subproblem is
// reversed through its K projected steps (masks 1[V > 0], the momentum
// weights, the step 1/L with dL = v^T dW v for the top eigenvector v), its
// small products, then the bases through the thin-QR adjoint and the X
// products.  X enters only through products X A and X^T B, so
// dL/dX = sum_j U_j V_j^T over 2(2q+1) rank-l pairs, formed by one final
// U V^T product.
#include <cmath>
#include <initializer_list>
#include <vector>

#include "ctx.hpp"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxK = 8;   // inner steps per subproblem the reverse supports

// ---------------------------------------------------------------------------
// Small dense products C = alpha op(A) op(B) + beta C (row-major), for the
// p x p, p x l, l x l, n x l, l x m shapes of the reverse pass.  Short
// reductions: one thread per output; long ones: one wavefront per output.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float opA(const float* A, int64_t lda, int ta, int64_t i, int64_t k) {
    return ta ? A[k * lda + i] : A[i * lda + k];
}
__device__ __forceinline__ float opB(const float* B, int64_t ldb, int tb, int64_t k, int64_t j) {
    return tb ? B[j * ldb + k] : B[k * ldb + j];
}

__global__ __launch_bounds__(kThreads) void k_gemm_short(int64_t M, int64_t N, int64_t K,
                                                        float alpha, const float* A, int64_t lda,
                                                        int ta, const float* B, int64_t ldb,
                                                        int tb, float beta, float* C,
                                                        int64_t ldc) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= M * N) return;
    const int64_t i = e / N, j = e - i * N;
    float s = 0.f;
    for (int64_t k = 0; k < K; ++k) s = fmaf(opA(A, lda, ta, i, k), opB(B, ldb, tb, k, j), s);
    const float old = beta != 0.f ? C[i * ldc + j] : 0.f;
    C[i * ldc + j] = alpha * s + beta * old;
}

__global__ __launch_bounds__(kThreads) void k_gemm_long(int64_t M, int64_t N, int64_t K,
                                                       float alpha, const float* A, int64_t lda,
                                                       int ta, const float* B, int64_t ldb,
                                                       int tb, float beta, float* C,
                                                       int64_t ldc) {
    const int lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= M * N) return;   // uniform per wave
    const int64_t i = e / N, j = e - i * N;
    float s = 0.f;
    for (int64_t k = lane; k < K; k += 64) s = fmaf(opA(A, lda, ta, i, k), opB(B, ldb, tb, k, j), s);
    s = wave_sum(s);
    if (lane == 0) {
        const float old = beta != 0.f ? C[i * ldc + j] : 0.f;
        C[i * ldc + j] = alpha * s + beta * old;
    }
}

// Up to two independent outputs per launch, each a sum of up to three
// products: C = sum_t alpha_t op(A_t) op(B_t) + beta C.  An output with a
// long reduction (any K > 64) takes one wavefront per entry, otherwise one
// lane per entry; the waves of output 0 come first.
struct MTerm {
    const float* A;
    const float* B;
    int64_t lda, ldb, K;
    int ta, tb;
    float alpha;
};
struct MOut {
    float* C;
    int64_t M, N, ldc;
    float beta;
    int nterm, wide;
    MTerm term[3];
};
struct MGemm {
    MOut out[2];
    int64_t first1, waves;   // first wave of output 1, total waves
};

__device__ __forceinline__ void mgemm_out(const MOut& u, int64_t w, int lane) {
    if (u.wide) {
        const int64_t i = w / u.N, j = w - i * u.N;
        float s = 0.f;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (t >= u.nterm) break;
            const MTerm& m = u.term[t];
            float acc = 0.f;
#pragma unroll 8
            for (int64_t k = lane; k < m.K; k += 64)
                acc = fmaf(opA(m.A, m.lda, m.ta, i, k), opB(m.B, m.ldb, m.tb, k, j), acc);
            s = fmaf(m.alpha, wave_sum(acc), s);
        }
        if (lane == 0) {
            const float old = u.beta != 0.f ? u.C[i * u.ldc + j] : 0.f;
            u.C[i * u.ldc + j] = fmaf(u.beta, old, s);
        }
    } else {
        const int64_t e = w * 64 + lane;
        if (e >= u.M * u.N) return;
        const int64_t i = e / u.N, j = e - i * u.N;
        float s = 0.f;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (t >= u.nterm) break;
            const MTerm& m = u.term[t];
            float acc = 0.f;
#pragma unroll 8
            for (int64_t k = 0; k < m.K; ++k)
                acc = fmaf(opA(m.A, m.lda, m.ta, i, k), opB(m.B, m.ldb, m.tb, k, j), acc);
            s = fmaf(m.alpha, acc, s);
        }
        const float old = u.beta != 0.f ? u.C[i * u.ldc + j] : 0.f;
        u.C[i * u.ldc + j] = fmaf(u.beta, old, s);
    }
}

__global__ __launch_bounds__(kThreads) void k_mgemm(MGemm g) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= g.waves) return;   // uniform per wave
    if (w < g.first1) mgemm_out(g.out[0], w, lane);
    else mgemm_out(g.out[1], w - g.first1, lane);
}

__global__ __launch_bounds__(kThreads) void k_axpy(int64_t n, float alpha, const float* x, float* y) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e < n) y[e] += alpha * x[e];
}

// dst (rows x cols, ldd) = src (rows x cols, lds)
__global__ __launch_bounds__(kThreads) void k_copy2d(int64_t rows, int64_t cols, const float* src,
                                                    int64_t lds, float* dst, int64_t ldd) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= rows * cols) return;
    const int64_t r = e / cols, c = e - r * cols;
    dst[r * ldd + c] = src[r * lds + c];
}

__global__ __launch_bounds__(kThreads) void k_fill_f(int64_t n, float v, float* y) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e < n) y[e] = v;
}

// C = tril(M) + tril(M, -1)^T  (l x l)
__global__ __launch_bounds__(kThreads) void k_copyltu(int l, const float* M, float* C) {
    for (int e = threadIdx.x; e < l * l; e += kThreads) {
        const int i = e / l, j = e % l;
        C[e] = i >= j ? M[i * l + j] : M[j * l + i];
    }
}

// Ri = R^-1 for the upper triangle of R (l x l), FP64, lane c owns column c.
__global__ __launch_bounds__(64) void k_tri_inv(int l, const float* R, float* Ri) {
    __shared__ double sR[32][33];
    for (int e = threadIdx.x; e < l * l; e += 64) sR[e / l][e % l] = (double)R[e];
    __syncthreads();
    const int c = threadIdx.x;
    if (c < l) {
        double x[32];
        for (int i = 0; i < 32; ++i) x[i] = 0.0;
        for (int i = l - 1; i >= 0; --i) {
            if (i > c) continue;
            double s = i == c ? 1.0 : 0.0;
            for (int t = i + 1; t <= c; ++t) s -= sR[i][t] * x[t];
            x[i] = s / sR[i][i];
        }
        for (int i = 0; i < l; ++i) Ri[i * l + c] = (float)x[i];
    }
}

// Unit eigenvector of the symmetric p x p W for its largest eigenvalue L, by
// two steps of inverse iteration with the shift sigma = L (1 + 1e-9) in
// FP64.  L is an upper bound of lambda_max, so W - sigma I is negative
// definite and Gaussian elimination without pivoting is stable; one
// wavefront, lane i keeps row i in registers, the pivot row of step k is
// read from lane k.  The sign is fixed so that the largest component is
// positive.
template <int P>
__global__ __launch_bounds__(64) void k_eigvec(int p, const float* Ws, const double* Ls, float* vs) {
    // workgroup b: W = Ws + b p^2, L = Ls[b], v = vs + 32 b
    const float* W = Ws + (int64_t)blockIdx.x * p * p;
    float* v = vs + (int64_t)blockIdx.x * 32;
    const int lane = threadIdx.x;
    const double L = Ls[blockIdx.x];
    const double sigma = L * (1.0 + 1e-9) + 1e-300;
    double x = lane < p ? 1.0 / sqrt((double)p) : 0.0;
    for (int it = 0; it < 2; ++it) {
        double R[P];
#pragma unroll
        for (int c = 0; c < P; ++c)
            R[c] = (lane < p && c < p)
                       ? 0.5 * ((double)W[lane * p + c] + (double)W[c * p + lane]) - (lane == c ? sigma : 0.0)
                       : (lane == c ? 1.0 : 0.0);
        double inv_own = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double dk = lane_d(R[k], k);
            if (dk == 0.0) dk = -1e-300;
            const double inv = 1.0 / dk;
            if (lane == k) inv_own = inv;
            const double f = (lane > k && lane < P) ? R[k] * inv : 0.0;
            x = fma(-f, lane_d(x, k), x);
#pragma unroll
            for (int c = k + 1; c < P; ++c) R[c] = fma(-f, lane_d(R[c], k), R[c]);
        }
        // back substitution: lane i keeps row i of the upper factor
        double xi = 0.0, acc = x;
#pragma unroll
        for (int k = P - 1; k >= 0; --k) {
            const double xk = lane_d(acc * inv_own, k);
            if (lane == k) xi = xk;
            if (lane < k) acc = fma(-R[k], xk, acc);
        }
        x = lane < p ? xi : 0.0;
        const double nrm = sqrt(wave_sum(x * x));
        x = nrm > 0.0 ? x / nrm : 0.0;
    }
    // sign: the component of largest magnitude positive (first of ties)
    const double ax = lane < p ? fabs(x) : -1.0;
    const double mx = wave_max(ax);
    const unsigned long long at = __ballot(lane < p && ax == mx);
    const int big = at ? __ffsll((long long)at) - 1 : 0;
    const double sg = lane_d(x, big) < 0.0 ? -1.0 : 1.0;
    if (lane < p) v[lane] = (float)(sg * x);
}

// ---------------------------------------------------------------------------
// Reverse of one Nesterov subproblem over `rows` independent rows (Sec. 2):
//   Y_k = Z_{k-1} + b_k (Z_{k-1} - Z_{k-2})   (Z_{-1} = Z_0, b_1 = b_2 = 0)
//   V_k = Y_k - (Y_k W - b) / L,   Z_k = max(0, V_k),   k = 1..K.
// Given Zbar = dL/dZ_K: Z0bar, Bbar (per row), and per-workgroup partials of
// Wbar = -(1/L) sum_k Y_k^T Vbar_k (before the 1/L) and of
// Lbar = sum_k <Vbar_k, Y_k - V_k> / L.  One wavefront per workgroup, one
// row per lane; the p x p partial of Y_k^T Vbar_k over the wavefront's 64
// rows is formed through LDS at every step, in FP64 and in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kAdjRows = 64;   // rows (lanes) per workgroup of the NNLS reverse
struct AdjNnls {
    int64_t rows;
    int p, K;
    const float* Z0;
    int64_t z_rs, z_cs;
    const float* W;
    const float* B;
    int64_t b_rs, b_cs;
    const double* L;
    const float* Zbar;
    float* Z0bar;            // same strides as Z0
    float* Bbar;             // same strides as B
    double* Wpart;           // [gridDim.x][p][p]
    double* Lpart;           // [gridDim.x]
    float* Zs;               // P = 32: [K + 1][gridDim.x * kAdjRows][32] (HBM tape)
    float beta[kMaxK + 1];   // beta[k] = b_k, k = 1..K
};

// The iterates Z_0 .. Z_K of the workgroup's rows stay in LDS for P = 16
// (dynamic LDS of the bytes below, at most 40 KB) and go to an HBM tape for
// P = 32, where they would not fit beside the other arrays in 64 KB.
constexpr bool adj_lds_tape(int P) { return P <= 16; }
constexpr size_t adj_lds_bytes(int P, int K) {
    return adj_lds_tape(P) ? (size_t)(K + 1) * kAdjRows * (P + 1) * 4 : 0;
}

// g = y W - b for one row (W zero-padded to P x P in LDS, read as float4)
template <int P>
__device__ __forceinline__ void row_times_w(const float (&y)[P], const float (*sW)[P], float (&g)[P]) {
#pragma unroll
    for (int d = 0; d < P; ++d) {
        const float4* w4 = reinterpret_cast<const float4*>(sW[d]);
#pragma unroll
        for (int c4 = 0; c4 < P / 4; ++c4) {
            const float4 w = w4[c4];
            g[4 * c4 + 0] = fmaf(y[d], w.x, g[4 * c4 + 0]);
            g[4 * c4 + 1] = fmaf(y[d], w.y, g[4 * c4 + 1]);
            g[4 * c4 + 2] = fmaf(y[d], w.z, g[4 * c4 + 2]);
            g[4 * c4 + 3] = fmaf(y[d], w.w, g[4 * c4 + 3]);
        }
    }
}

template <int P>
__global__ __launch_bounds__(kAdjRows) void k_nnls_adj(AdjNnls a) {
    constexpr int NE = (P * P + kAdjRows - 1) / kAdjRows;   // W entries per lane
    __shared__ __align__(16) float sW[P][P];
    __shared__ float sy[kAdjRows][P + 1], sv[kAdjRows][P + 1];
    extern __shared__ float zt[];   // [K + 1][kAdjRows][P + 1]
    const int p = a.p;
    const int lane = threadIdx.x;
    for (int e = lane; e < P * P; e += kAdjRows) {
        const int d = e / P, c = e % P;
        sW[d][c] = (d < p && c < p) ? a.W[d * p + c] : 0.f;
    }
    __syncthreads();
    const double Ld = *a.L;
    const float invL = (float)(1.0 / Ld);
    const int64_t r = (int64_t)blockIdx.x * kAdjRows + lane;
    const bool valid = r < a.rows;
    auto zs = [&](int k) -> float* {
        if constexpr (adj_lds_tape(P)) return zt + ((size_t)k * kAdjRows + lane) * (P + 1);
        else return a.Zs + ((int64_t)k * gridDim.x * kAdjRows + r) * 32;
    };
    // rows past the end run on zeros: every product below is then zero
    float b[P], zc[P], zp[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        b[c] = (valid && c < p) ? a.B[r * a.b_rs + c * a.b_cs] : 0.f;
        zc[c] = (valid && c < p) ? a.Z0[r * a.z_rs + c * a.z_cs] : 0.f;
        zp[c] = zc[c];
    }
#pragma unroll
    for (int c = 0; c < P; ++c) zs(0)[c] = zc[c];
    // forward recompute, keeping Z_0 .. Z_K
    for (int k = 1; k <= a.K; ++k) {
        const float bk = a.beta[k];
        float y[P], g[P];
#pragma unroll
        for (int c = 0; c < P; ++c) {
            y[c] = fmaf(bk, zc[c] - zp[c], zc[c]);
            g[c] = -b[c];
        }
        row_times_w<P>(y, sW, g);
#pragma unroll
        for (int c = 0; c < P; ++c) {
            const float v = fmaf(-g[c], invL, y[c]);
            zp[c] = zc[c];
            zc[c] = (v > 0.f || v != v) ? v : 0.f;
            zs(k)[c] = zc[c];
        }
    }
    // reverse: za = dL/dZ_k (complete), zb = dL/dZ_{k-1}, zq = dL/dZ_{k-2}
    float za[P], zb[P], zq[P], bb[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        za[c] = (valid && c < p) ? a.Zbar[r * a.z_rs + c * a.z_cs] : 0.f;
        zb[c] = 0.f;
        zq[c] = 0.f;
        bb[c] = 0.f;
    }
    double wacc[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) wacc[j] = 0.0;
    double lbar = 0.0;
    for (int k = a.K; k >= 1; --k) {
        const float bk = a.beta[k];
        const float* z1 = zs(k - 1);
        const float* z2 = zs(k >= 2 ? k - 2 : 0);
        float y[P], g[P], vb[P];
#pragma unroll
        for (int c = 0; c < P; ++c) {
            y[c] = fmaf(bk, z1[c] - z2[c], z1[c]);
            g[c] = -b[c];
        }
        row_times_w<P>(y, sW, g);
#pragma unroll
        for (int c = 0; c < P; ++c) {
            const float v = fmaf(-g[c], invL, y[c]);
            vb[c] = (v > 0.f) ? za[c] : 0.f;
            lbar += (double)vb[c] * (double)(y[c] - v);
        }
        // this step's Y^T Vbar over the workgroup's rows
        __syncthreads();
#pragma unroll
        for (int c = 0; c < P; ++c) {
            sy[lane][c] = y[c];
            sv[lane][c] = vb[c];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            const int e = lane + j * kAdjRows;
            if (e < p * p) {
                const int dd = e / p, cc = e - dd * p;
                double s = 0.0;
                for (int rr = 0; rr < kAdjRows; ++rr) s = fma((double)sy[rr][dd], (double)sv[rr][cc], s);
                wacc[j] += s;
            }
        }
        // ybar = vbar (I - W / L)^T, with V = Y (I - W/L) + b / L; W is
        // symmetric, so vbar W^T = vbar W
        float s[P];
#pragma unroll
        for (int c = 0; c < P; ++c) s[c] = 0.f;
        row_times_w<P>(vb, sW, s);
#pragma unroll
        for (int c = 0; c < P; ++c) {
            const float yb = fmaf(-s[c], invL, vb[c]);
            bb[c] = fmaf(vb[c], invL, bb[c]);
            if (k >= 2) {
                zb[c] = fmaf(1.f + bk, yb, zb[c]);
                zq[c] = fmaf(-bk, yb, zq[c]);
            } else {
                zb[c] += yb;   // Z_{-1} is Z_0
            }
        }
#pragma unroll
        for (int c = 0; c < P; ++c) {
            za[c] = zb[c];
            zb[c] = zq[c];
            zq[c] = 0.f;
        }
    }
    if (valid)
        for (int c = 0; c < p; ++c) {
            a.Z0bar[r * a.z_rs + c * a.z_cs] = za[c];
            a.Bbar[r * a.b_rs + c * a.b_cs] = bb[c];
        }
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        const int e = lane + j * kAdjRows;
        if (e < p * p) a.Wpart[(int64_t)blockIdx.x * p * p + e] = wacc[j];
    }
    lbar = wave_sum(lbar / Ld);
    if (lane == 0) a.Lpart[blockIdx.x] = lbar;
}

// Wbs = Wbar + Wbar^T with Wbar[d][c] = -(1/L) sum_b Wpart[b][d][c] +
// Lbar v_d v_c, Lbar = sum of the Lpart; both sums in workgroup order (the
// partials of eight workgroups loaded together).
__global__ __launch_bounds__(kThreads) void k_wbar(int p, const double* Wpart, const double* Lpart,
                                                  int nparts, const double* Lp, const float* v,
                                                  float* Wbs) {
    __shared__ double slb;
    __shared__ float sw[32][33];
    if (threadIdx.x < 64) {
        double lb = 0.0;
        for (int k = threadIdx.x; k < nparts; k += 64) lb += Lpart[k];
        lb = wave_sum(lb);
        if (threadIdx.x == 0) slb = lb;
    }
    __syncthreads();
    const int64_t pp = (int64_t)p * p;
    for (int e = threadIdx.x; e < pp; e += kThreads) {
        const int d = e / p, c = e % p;
        double s = 0.0;
        int b = 0;
        for (; b + 8 <= nparts; b += 8) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = Wpart[(b + u) * pp + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += t[u];
        }
        for (; b < nparts; ++b) s += Wpart[b * pp + e];
        sw[d][c] = (float)(-s / *Lp + slb * (double)v[d] * (double)v[c]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < pp; e += kThreads) {
        const int d = e / p, c = e % p;
        Wbs[e] = sw[d][c] + sw[c][d];
    }
}

// dX (n x m, ldd) = U V^T with U n x r, V m x r (row-major): 64 x 64 tiles,
// 4 x 4 outputs per thread, reduction staged through LDS in chunks of 16.
__global__ __launch_bounds__(kThreads) void k_gemm_nt(int64_t n, int64_t m, int r, const float* U,
                                                     const float* V, float* dX, int64_t ldd) {
    __shared__ float su[16][68], sv[16][68];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
    for (int k0 = 0; k0 < r; k0 += 16) {
        __syncthreads();
        for (int e = threadIdx.x; e < 16 * 64; e += kThreads) {
            const int kk = e % 16, rr = e / 16;
            const int64_t iu = i0 + rr, jv = j0 + rr;
            const int k = k0 + kk;
            su[kk][rr] = (iu < n && k < r) ? U[iu * r + k] : 0.f;
            sv[kk][rr] = (jv < m && k < r) ? V[jv * r + k] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a4[4], b4[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) a4[a] = su[kk][ty * 4 + a];
#pragma unroll
            for (int b = 0; b < 4; ++b) b4[b] = sv[kk][tx * 4 + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(a4[a], b4[b], acc[a][b]);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t i = i0 + ty * 4 + a, j = j0 + tx * 4 + b;
            if (i < n && j < m) dX[i * ldd + j] = acc[a][b];
        }
}

unsigned nb(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct cnmf_tape {
    cnmf_ctx* c = nullptr;
    int64_t n = 0, m = 0, ldx = 0, ldt = 0;
    int p = 0, l = 0, q = 0, T = 0, K = 0, ck = 0;
    const float* X = nullptr;
    const float* oL = nullptr;
    const float* oR = nullptr;
    char* mem = nullptr;
    size_t bytes = 0;
    // RSI tape (see rsi_forward)
    float *oRt = nullptr, *oLT = nullptr;
    std::vector<float*> A, QL, Cn, QtRt;        // n x l panels
    std::vector<float*> Bm, QRt, Cm, QtL;       // m x l panels
    std::vector<float*> QRtT, QtLT;             // transposes, l x ldt
    float *QLo = nullptr, *QRo = nullptr, *XL = nullptr, *XR = nullptr;   // compressed data
    // checkpoints and segment recompute
    std::vector<float*> Gc, Fc;                 // (G, F) at t = 0, ck, 2 ck, ...
    float *Gh = nullptr, *Fh = nullptr;         // ck x n x p, ck x p x m
    float* Wh = nullptr;                        // ck x 2 x p x p: each subproblem's W
    float* Vh = nullptr;                        // ck x 2 x 32: its top eigenvector
    double* Lh = nullptr;                       // ck x 2: each subproblem's L
    int32_t* replay = nullptr;                  // T x 2, all K
    int32_t* rep = nullptr;                     // 4q x 32 replaced-column flags of the RSI
    float* part = nullptr;                      // sweep partials
    // reverse work buffers
    float *Gb = nullptr, *Fb = nullptr, *Gb2 = nullptr, *Fb2 = nullptr;
    float *XRb = nullptr, *XLb = nullptr, *QLb = nullptr, *QRb = nullptr;
    float *GL = nullptr, *FR = nullptr, *Bsub = nullptr, *Bsub2 = nullptr, *Bb = nullptr, *Wb = nullptr;
    float *GLb = nullptr, *FRb = nullptr;
    double *Wpart = nullptr, *Lpart = nullptr;
    float* Zs = nullptr;                        // p > 16: HBM tape of the NNLS reverse
    float *U = nullptr, *V = nullptr;           // n x r, m x r
    float *Tn = nullptr, *Tm = nullptr, *Tn2 = nullptr, *Tm2 = nullptr;   // panel temporaries
    float *Rl = nullptr, *Ril = nullptr, *Ml = nullptr, *Cl = nullptr;   // l x l
    std::vector<float*> QLb_k, QRtb_k;          // adjoints of QL_k, QRt_k (k < q)
};

namespace {

hipError_t gemm(const Dev& d, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                int64_t lda, bool ta, const float* B, int64_t ldb, bool tb, float beta, float* C,
                int64_t ldc) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K > 64)
        hipLaunchKernelGGL(k_gemm_long, dim3(nb(M * N, 4)), dim3(kThreads), 0, d.stream, M, N, K,
                           alpha, A, lda, ta ? 1 : 0, B, ldb, tb ? 1 : 0, beta, C, ldc);
    else
        hipLaunchKernelGGL(k_gemm_short, dim3(nb(M * N, kThreads)), dim3(kThreads), 0, d.stream, M,
                           N, K, alpha, A, lda, ta ? 1 : 0, B, ldb, tb ? 1 : 0, beta, C, ldc);
    return hipGetLastError();
}

MTerm term(const float* A, int64_t lda, bool ta, const float* B, int64_t ldb, bool tb, int64_t K,
           float alpha = 1.f) {
    MTerm m{};
    m.A = A;
    m.B = B;
    m.lda = lda;
    m.ldb = ldb;
    m.K = K;
    m.ta = ta ? 1 : 0;
    m.tb = tb ? 1 : 0;
    m.alpha = alpha;
    return m;
}

MOut out(float* C, int64_t M, int64_t N, int64_t ldc, float beta, std::initializer_list<MTerm> ts) {
    MOut o{};
    o.C = C;
    o.M = M;
    o.N = N;
    o.ldc = ldc;
    o.beta = beta;
    for (const MTerm& m : ts) {
        o.term[o.nterm++] = m;
        if (m.K > 64) o.wide = 1;
    }
    return o;
}

int64_t out_waves(const MOut& o) { return o.wide ? o.M * o.N : (o.M * o.N + 63) / 64; }

// o0 and o1 in one launch (independent outputs)
hipError_t mgemm(const Dev& d, const MOut& o0, const MOut& o1) {
    MGemm g{};
    g.out[0] = o0;
    g.out[1] = o1;
    g.first1 = out_waves(o0);
    g.waves = g.first1 + out_waves(o1);
    if (g.waves <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mgemm, dim3(nb(g.waves, 4)), dim3(kThreads), 0, d.stream, g);
    return hipGetLastError();
}

hipError_t axpy(const Dev& d, int64_t n, float alpha, const float* x, float* y) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy, dim3(nb(n, kThreads)), dim3(kThreads), 0, d.stream, n, alpha, x, y);
    return hipGetLastError();
}

hipError_t fillf(const Dev& d, int64_t n, float v, float* y) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f, dim3(nb(n, kThreads)), dim3(kThreads), 0, d.stream, n, v, y);
    return hipGetLastError();
}

hipError_t copy2d(const Dev& d, int64_t rows, int64_t cols, const float* src, int64_t lds,
                  float* dst, int64_t ldd) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy2d, dim3(nb(rows * cols, kThreads)), dim3(kThreads), 0, d.stream,
                       rows, cols, src, lds, dst, ldd);
    return hipGetLastError();
}

#define HK(x)                                   \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

// Thin-QR adjoint of Q = qr(Y) (R unused downstream), N x l panels:
//   M = -Qbar^T Q,  Ybar = (Qbar + Q copyltu(M)) R^-T,  R = Q^T Y.
hipError_t orth_adj(cnmf_tape* t, const Dev& d, int64_t N, const float* Y, const float* Q,
                    const float* Qb, float* Yb, float* tmp) {
    const int l = t->l;
    HK(gemm(d, l, l, N, 1.f, Q, l, true, Y, l, false, 0.f, t->Rl, l));
    HK(gemm(d, l, l, N, -1.f, Qb, l, true, Q, l, false, 0.f, t->Ml, l));
    hipLaunchKernelGGL(k_copyltu, dim3(1), dim3(kThreads), 0, d.stream, l, t->Ml, t->Cl);
    HK(hipGetLastError());
    hipLaunchKernelGGL(k_tri_inv, dim3(1), dim3(64), 0, d.stream, l, t->Rl, t->Ril);
    HK(hipGetLastError());
    HK(copy2d(d, N, l, Qb, l, tmp, l));
    HK(gemm(d, N, l, l, 1.f, Q, l, false, t->Cl, l, false, 1.f, tmp, l));
    return gemm(d, N, l, l, 1.f, tmp, l, false, t->Ril, l, true, 0.f, Yb, l);
}

// Forward randomized subspace iteration keeping every panel (Algorithm 2,
// the same chain and kernels as the plain entry point).
int rsi_forward(cnmf_tape* t) {
    cnmf_ctx* c = t->c;
    const Dev& d = c->dev;
    const int64_t n = t->n, m = t->m;
    const int l = t->l, q = t->q;
    const double tau2 = 1e-9;
    int nrep = 0;   // every orthonormalisation records its replaced columns
    auto orth_n = [&](const float* Y, float* Q) -> hipError_t {
        unsigned seq = 0;
        HK(next_seq(c, &seq));
        return orth(d, n, l, Y, t->oRt, false, tau2, Q, nullptr, 0, t->rep + 32 * nrep++, c->oxch,
                    seq, c->ctl);
    };
    auto orth_m = [&](const float* Y, float* Q, float* QT) -> hipError_t {
        unsigned seq = 0;
        HK(next_seq(c, &seq));
        return orth(d, m, l, Y, t->oL, false, tau2, Q, QT, t->ldt, t->rep + 32 * nrep++, c->oxch,
                    seq, c->ctl);
    };
    auto right = [&](const float* AT, float* Y) {
        return sweep_right(d, n, m, t->X, t->ldx, l, AT, t->ldt, true, Y, l, t->part);
    };
    auto left = [&](const float* B, float* Z) {
        return sweep_left(d, n, m, t->X, t->ldx, l, B, l, Z, l, false, t->part);
    };
    CK(transpose(d, l, n, t->oR, n, t->oRt, l));
    CK(transpose(d, m, l, t->oL, l, t->oLT, t->ldt));
    CK(right(t->oLT, t->A[0]));
    CK(orth_n(t->A[0], t->QL[0]));
    CK(left(t->oRt, t->Bm[0]));
    CK(orth_m(t->Bm[0], t->QRt[0], t->QRtT[0]));
    for (int k = 1; k <= q; ++k) {
        CK(left(t->QL[k - 1], t->Cm[k]));
        CK(orth_m(t->Cm[k], t->QtL[k], t->QtLT[k]));
        CK(right(t->QRtT[k - 1], t->Cn[k]));
        CK(orth_n(t->Cn[k], t->QtRt[k]));
        CK(right(t->QtLT[k], t->A[k]));
        CK(left(t->QtRt[k], t->Bm[k]));
        if (k < q) {
            CK(orth_n(t->A[k], t->QL[k]));
            CK(orth_m(t->Bm[k], t->QRt[k], t->QRtT[k]));
        }
    }
    // compressed data: Q_L = Q~_R^(q)^T panel, Q_R = Q~_L^(q), X_R = A_q, X_L = B_q^T
    t->QLo = t->QtRt[q];
    t->QRo = t->QtL[q];
    t->XR = t->A[q];
    CK(transpose(d, m, l, t->Bm[q], l, t->XL, m));
    return CNMF_OK;
}

// Outer iterations [t0, t0 + cnt) from (G, F) in place; with hist, every
// iterate and every subproblem's W and L are kept (segment recompute).
int solve_span(cnmf_tape* t, float* G, float* F, int t0, int cnt, bool hist) {
    cnmf_params prm;
    cnmf_params_default(&prm);
    prm.p = t->p;
    prm.nu = t->l - t->p;
    prm.q = t->q;
    prm.outer_iters = cnt;
    prm.inner_max = t->K;
    prm.stop_rule = CNMF_STOP_SUBPROBLEM;
    cnmf_trace tr{};
    if (hist) {
        tr.G_hist = t->Gh;
        tr.F_hist = t->Fh;
        tr.W_hist = t->Wh;
        tr.lips = t->Lh;
    }
    return cnmf_solve(t->c, CNMF_METHOD_COMPRESSED, t->n, t->m, nullptr, 0, t->QLo, t->QRo, t->XL,
                      t->XR, &prm, G, F, hist ? &tr : nullptr, t->replay + 2 * t0);
}

// Reverse of one subproblem: Zbar (adjoint of its output) -> Z0bar, and the
// adjoints of its W, B and L folded into Wb (p x p, W's adjoint plus its
// transpose) and Bb (strided like B).  W, L and the top eigenvector v are
// the forward's (kept by the recompute).
int subproblem_adj(cnmf_tape* t, const Dev& d, int64_t rows, const float* W, const double* L,
                   const float* v, const float* Z0, int64_t z_rs, int64_t z_cs, const float* B,
                   int64_t b_rs, int64_t b_cs, const float* Zbar, float* Z0bar) {
    const int p = t->p;
    AdjNnls a{};
    a.rows = rows;
    a.p = p;
    a.K = t->K;
    a.Z0 = Z0;
    a.z_rs = z_rs;
    a.z_cs = z_cs;
    a.W = W;
    a.B = B;
    a.b_rs = b_rs;
    a.b_cs = b_cs;
    a.L = L;
    a.Zbar = Zbar;
    a.Z0bar = Z0bar;
    a.Bbar = t->Bb;
    a.Wpart = t->Wpart;
    a.Lpart = t->Lpart;
    a.Zs = t->Zs;
    // momentum weights of the forward kernel (the same table): step k uses beta[k]
    {
        float tab[kMaxK + 1];
        momentum_table(tab, t->K);
        a.beta[0] = 0.f;
        for (int k = 1; k <= t->K; ++k) a.beta[k] = tab[k - 1];
    }
    // one wavefront per workgroup: the rows' serial chains spread over many
    // compute units instead of sharing four per unit
    const unsigned blocks = nb(rows, kAdjRows);
    if (p <= 16)
        hipLaunchKernelGGL(k_nnls_adj<16>, dim3(blocks), dim3(kAdjRows), adj_lds_bytes(16, t->K),
                           d.stream, a);
    else
        hipLaunchKernelGGL(k_nnls_adj<32>, dim3(blocks), dim3(kAdjRows), adj_lds_bytes(32, t->K),
                           d.stream, a);
    CK(hipGetLastError());
    hipLaunchKernelGGL(k_wbar, dim3(1), dim3(kThreads), 0, d.stream, p, t->Wpart, t->Lpart,
                       (int)blocks, L, v, t->Wb);
    CK(hipGetLastError());
    return CNMF_OK;
}

// Reverse of outer iteration t (entry j of the recomputed segment): (Gb, Fb)
// hold dL/dG_t, dL/dF_t on entry and dL/dG_{t-1}, dL/dF_{t-1} on exit; the
// compressed-data adjoints accumulate.  G_t = NNLS(G_{t-1}; F_R F_R^T,
// X_R F_R^T) with F_R = F_{t-1} Q_R, then F_t = NNLS(F_{t-1}; G_L^T G_L,
// G_L^T X_L) with G_L = Q_L^T G_t; the F update is reversed first.
int outer_adj(cnmf_tape* t, int j, const float* Gprev, const float* Fprev, const float* Gcur) {
    const Dev& d = t->c->dev;
    const int64_t n = t->n, m = t->m;
    const int p = t->p, l = t->l;
    const size_t pp = (size_t)p * p;
    const int sG = 2 * j, sF = 2 * j + 1;   // subproblem slots in the kept W, L, v
    // G_L = Q_L^T G_t (l x p) and F_R = F_{t-1} Q_R (p x l)
    CK(mgemm(d, out(t->GL, l, p, p, 0.f, {term(t->QLo, l, true, Gcur, p, false, n)}),
             out(t->FR, p, l, l, 0.f, {term(Fprev, m, false, t->QRo, l, false, m)})));
    // the subproblems' B: G_L^T X_L (p x m) and X_R F_R^T (n x p)
    CK(mgemm(d, out(t->Bsub, p, m, m, 0.f, {term(t->GL, p, true, t->XL, m, false, l)}),
             out(t->Bsub2, n, p, p, 0.f, {term(t->XR, l, false, t->FR, l, true, l)})));
    // ---- F update
    int rc = subproblem_adj(t, d, m, t->Wh + sF * pp, t->Lh + sF, t->Vh + 32 * sF, Fprev, 1, m,
                            t->Bsub, 1, m, t->Fb, t->Fb2);
    if (rc) return rc;
    // G_L bar = G_L Wb + X_L Bb^T ; X_L bar += G_L Bb
    CK(mgemm(d, out(t->GLb, l, p, p, 0.f, {term(t->GL, p, false, t->Wb, p, false, p),
                                           term(t->XL, m, false, t->Bb, m, true, m)}),
             out(t->XLb, l, m, m, 1.f, {term(t->GL, p, false, t->Bb, m, false, p)})));
    // G_t bar += Q_L G_L bar ; Q_L bar += G_t G_L bar^T
    CK(mgemm(d, out(t->Gb, n, p, p, 1.f, {term(t->QLo, l, false, t->GLb, p, false, l)}),
             out(t->QLb, n, l, l, 1.f, {term(Gcur, p, false, t->GLb, p, true, p)})));
    // ---- G update
    rc = subproblem_adj(t, d, n, t->Wh + sG * pp, t->Lh + sG, t->Vh + 32 * sG, Gprev, p, 1,
                        t->Bsub2, p, 1, t->Gb, t->Gb2);
    if (rc) return rc;
    // F_R bar = Wb F_R + Bb^T X_R ; X_R bar += Bb F_R
    CK(mgemm(d, out(t->FRb, p, l, l, 0.f, {term(t->Wb, p, false, t->FR, l, false, p),
                                           term(t->Bb, p, true, t->XR, l, false, n)}),
             out(t->XRb, n, l, l, 1.f, {term(t->Bb, p, false, t->FR, l, false, p)})));
    // F_{t-1} bar += F_R bar Q_R^T ; Q_R bar += F_{t-1}^T F_R bar
    CK(mgemm(d, out(t->Fb2, p, m, m, 1.f, {term(t->FRb, l, false, t->QRo, l, true, l)}),
             out(t->QRb, m, l, l, 1.f, {term(Fprev, m, true, t->FRb, l, false, p)})));
    std::swap(t->Gb, t->Gb2);
    std::swap(t->Fb, t->Fb2);
    return CNMF_OK;
}

// Reverse of Algorithm 2 from the compressed-data adjoints; the rank-l pairs
// of dL/dX go to columns of U (n x r) and V (m x r).
int rsi_adj(cnmf_tape* t) {
    const Dev& d = t->c->dev;
    const int64_t n = t->n, m = t->m;
    const int l = t->l, q = t->q;
    const int r = 2 * (2 * q + 1) * l;
    int col = 0;
    auto pair = [&](const float* Up, const float* Vp) -> hipError_t {
        HK(copy2d(d, n, l, Up, l, t->U + col, r));
        HK(copy2d(d, m, l, Vp, l, t->V + col, r));
        col += l;
        return hipSuccess;
    };
    auto right = [&](const float* A, float* Y) {   // Y = X A, A m x l
        return sweep_right(d, n, m, t->X, t->ldx, l, A, l, false, Y, l, t->part);
    };
    auto left = [&](const float* B, float* Z) {    // Z = X^T B, B n x l
        return sweep_left(d, n, m, t->X, t->ldx, l, B, l, Z, l, false, t->part);
    };
    // adjoints of X_R (= A_q) and X_L^T (= B_q)
    float* Ab = t->XRb;
    CK(transpose(d, l, m, t->XLb, m, t->Tm2, l));   // Bb_q (m x l)
    float* Bb = t->Tm2;
    float* QtRtb = t->QLb;   // dL/dQ~_R^(q) panel = dL/dQ_L
    float* QtLb = t->QRb;    // dL/dQ~_L^(q) = dL/dQ_R
    for (int k = q; k >= 1; --k) {
        if (k < q) {
            // A_k -> QL_k, B_k -> QRt_k
            CK(orth_adj(t, d, n, t->A[k], t->QL[k], t->QLb_k[k], t->Tn2, t->Tn));
            Ab = t->Tn2;
            CK(orth_adj(t, d, m, t->Bm[k], t->QRt[k], t->QRtb_k[k], t->Tm2, t->Tm));
            Bb = t->Tm2;
            // the bases of this half-step start from zero
            CK(fillf(d, n * l, 0.f, t->QLb));
            CK(fillf(d, m * l, 0.f, t->QRb));
            QtRtb = t->QLb;
            QtLb = t->QRb;
        }
        // B_k = X^T QtRt_k: pair (QtRt_k, Bb_k), QtRt_k bar += X Bb_k
        CK(pair(t->QtRt[k], Bb));
        CK(right(Bb, t->Tn));
        CK(axpy(d, n * l, 1.f, t->Tn, QtRtb));
        // A_k = X QtL_k: pair (Ab_k, QtL_k), QtL_k bar += X^T Ab_k
        CK(pair(Ab, t->QtL[k]));
        CK(left(Ab, t->Tm));
        CK(axpy(d, m * l, 1.f, t->Tm, QtLb));
        // QtRt_k = orth(Cn_k), Cn_k = X QRt_{k-1}
        CK(orth_adj(t, d, n, t->Cn[k], t->QtRt[k], QtRtb, t->Tn2, t->Tn));
        CK(pair(t->Tn2, t->QRt[k - 1]));
        CK(left(t->Tn2, t->QRtb_k[k - 1]));
        // QtL_k = orth(Cm_k), Cm_k = X^T QL_{k-1}
        CK(orth_adj(t, d, m, t->Cm[k], t->QtL[k], QtLb, t->Tm2, t->Tm));
        CK(pair(t->QL[k - 1], t->Tm2));
        CK(right(t->Tm2, t->QLb_k[k - 1]));
    }
    // step 0: QRt_0 = orth(B_0), B_0 = X^T Omega_R^T ; QL_0 = orth(A_0), A_0 = X Omega_L
    CK(orth_adj(t, d, m, t->Bm[0], t->QRt[0], t->QRtb_k[0], t->Tm2, t->Tm));
    CK(pair(t->oRt, t->Tm2));
    CK(orth_adj(t, d, n, t->A[0], t->QL[0], t->QLb_k[0], t->Tn2, t->Tn));
    CK(pair(t->Tn2, t->oL));
    return col == r ? CNMF_OK : CNMF_EINVAL;
}

}  // namespace

extern "C" {

int cnmf_adj_forward(cnmf_ctx* c, int64_t n, int64_t m, const float* X, int64_t ldx,
                     const cnmf_params* prm, int32_t ckpt, const float* omega_L,
                     const float* omega_R, const float* G0, const float* F0, float* G_out,
                     float* F_out, cnmf_tape** tape_out) {
    if (!c || !tape_out || !prm) return CNMF_EINVAL;
    *tape_out = nullptr;
    if (check_params(prm, n, m, true)) return CNMF_EINVAL;
    if (prm->p > 32 || prm->inner_max < 1 || prm->inner_max > kMaxK) return CNMF_EINVAL;
    if (ckpt < 1 || prm->outer_iters < 1) return CNMF_EINVAL;
    if (bad_ptr(X) || ldx < m || bad_ptr(omega_L) || bad_ptr(omega_R) || bad_ptr(G0) ||
        bad_ptr(F0) || bad_ptr(G_out) || bad_ptr(F_out))
        return CNMF_EINVAL;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    cnmf_tape* t = new (std::nothrow) cnmf_tape;
    if (!t) return CNMF_ENOMEM;
    t->c = c;
    t->n = n;
    t->m = m;
    t->X = X;
    t->ldx = ldx;
    t->oL = omega_L;
    t->oR = omega_R;
    t->p = prm->p;
    t->l = prm->p + prm->nu;
    t->q = prm->q;
    t->T = prm->outer_iters;
    t->K = prm->inner_max;
    t->ck = ckpt;
    t->ldt = (m + 3) / 4 * 4;
    const int l = t->l, q = t->q, p = t->p, T = t->T;
    const int r = 2 * (2 * q + 1) * l;
    const int nck = (T + ckpt - 1) / ckpt + 1;
    Arena ar;
    std::vector<size_t> o;
    auto take = [&](size_t floats) { o.push_back(ar.take<float>(floats)); };
    const size_t NL = (size_t)n * l, ML = (size_t)m * l, LT = (size_t)l * t->ldt;
    take(NL);            // 0 oRt
    take(LT);            // 1 oLT
    for (int k = 0; k <= q; ++k) { take(NL); take(NL); take(NL); take(NL); }   // A, QL, Cn, QtRt
    for (int k = 0; k <= q; ++k) { take(ML); take(ML); take(ML); take(ML); }   // Bm, QRt, Cm, QtL
    for (int k = 0; k <= q; ++k) { take(LT); take(LT); }                       // QRtT, QtLT
    take((size_t)l * m);                                                       // XL
    for (int k = 0; k < nck; ++k) { take((size_t)n * p); take((size_t)p * m); }   // checkpoints
    take((size_t)ckpt * n * p);
    take((size_t)ckpt * p * m);
    take((size_t)ckpt * 2 * p * p);                                            // Wh
    take((size_t)ckpt * 2 * 32);                                               // Vh
    const size_t o_lh = ar.take<double>((size_t)ckpt * 2);
    const size_t o_rep = ar.take<int32_t>((size_t)2 * T);
    const size_t o_flags = ar.take<int32_t>((size_t)4 * q * 32);
    const size_t pf = std::max(sweep_right_partial_floats(c->dev, n, m),
                               sweep_left_partial_floats(c->dev, n, m));
    take(pf + 1);                                                              // part
    const size_t base_work = o.size();
    take((size_t)n * p); take((size_t)p * m); take((size_t)n * p); take((size_t)p * m);   // Gb Fb Gb2 Fb2
    take(NL); take((size_t)l * m); take(NL); take(ML);                         // XRb XLb QLb QRb
    take((size_t)l * p); take((size_t)p * l);                                  // GL FR
    const int64_t nm = std::max(n, m);
    take((size_t)nm * p); take((size_t)nm * p); take((size_t)nm * p);          // Bsub Bsub2 Bb
    take((size_t)p * p); take((size_t)l * p); take((size_t)p * l);             // Wb GLb FRb
    const size_t nm_pad = (size_t)nb(nm, kAdjRows) * kAdjRows;
    take(p > 16 ? (size_t)(kMaxK + 1) * nm_pad * 32 : 1);                      // Zs
    const size_t o_wp = ar.take<double>((size_t)nb(nm, kAdjRows) * p * p);
    const size_t o_lp = ar.take<double>(nb(nm, kAdjRows));
    take((size_t)n * r); take((size_t)m * r);                                  // U V
    take(NL); take(ML); take(NL); take(ML);                                    // Tn Tm Tn2 Tm2
    take((size_t)l * l); take((size_t)l * l); take((size_t)l * l); take((size_t)l * l);
    for (int k = 0; k < q; ++k) { take(NL); take(ML); }                        // QLb_k QRtb_k
    if (hipMalloc((void**)&t->mem, ar.off) != hipSuccess) {
        delete t;
        return CNMF_ENOMEM;
    }
    t->bytes = ar.off;
    auto F = [&](size_t i) { return reinterpret_cast<float*>(t->mem + o[i]); };
    size_t i = 0;
    t->oRt = F(i++);
    t->oLT = F(i++);
    t->A.resize(q + 1); t->QL.resize(q + 1); t->Cn.resize(q + 1); t->QtRt.resize(q + 1);
    for (int k = 0; k <= q; ++k) { t->A[k] = F(i++); t->QL[k] = F(i++); t->Cn[k] = F(i++); t->QtRt[k] = F(i++); }
    t->Bm.resize(q + 1); t->QRt.resize(q + 1); t->Cm.resize(q + 1); t->QtL.resize(q + 1);
    for (int k = 0; k <= q; ++k) { t->Bm[k] = F(i++); t->QRt[k] = F(i++); t->Cm[k] = F(i++); t->QtL[k] = F(i++); }
    t->QRtT.resize(q + 1); t->QtLT.resize(q + 1);
    for (int k = 0; k <= q; ++k) { t->QRtT[k] = F(i++); t->QtLT[k] = F(i++); }
    t->XL = F(i++);
    for (int k = 0; k < nck; ++k) { t->Gc.push_back(F(i++)); t->Fc.push_back(F(i++)); }
    t->Gh = F(i++);
    t->Fh = F(i++);
    t->Wh = F(i++);
    t->Vh = F(i++);
    t->Lh = reinterpret_cast<double*>(t->mem + o_lh);
    t->replay = reinterpret_cast<int32_t*>(t->mem + o_rep);
    t->rep = reinterpret_cast<int32_t*>(t->mem + o_flags);
    t->part = F(i++);
    if (i != base_work) { cnmf_tape_destroy(t); return CNMF_EINVAL; }
    t->Gb = F(i++); t->Fb = F(i++); t->Gb2 = F(i++); t->Fb2 = F(i++);
    t->XRb = F(i++); t->XLb = F(i++); t->QLb = F(i++); t->QRb = F(i++);
    t->GL = F(i++); t->FR = F(i++);
    t->Bsub = F(i++); t->Bsub2 = F(i++); t->Bb = F(i++);
    t->Wb = F(i++); t->GLb = F(i++); t->FRb = F(i++);
    t->Zs = F(i++);
    t->Wpart = reinterpret_cast<double*>(t->mem + o_wp);
    t->Lpart = reinterpret_cast<double*>(t->mem + o_lp);
    t->U = F(i++); t->V = F(i++);
    t->Tn = F(i++); t->Tm = F(i++); t->Tn2 = F(i++); t->Tm2 = F(i++);
    t->Rl = F(i++); t->Ril = F(i++); t->Ml = F(i++); t->Cl = F(i++);
    for (int k = 0; k < q; ++k) { t->QLb_k.push_back(F(i++)); t->QRtb_k.push_back(F(i++)); }
    const Dev& d = c->dev;
    const uint64_t kk = (uint64_t)(uint32_t)t->K;
    int rc = CNMF_OK;
    if (fill_u64(d, reinterpret_cast<uint64_t*>(t->replay), T, kk | (kk << 32)) != hipSuccess ||
        fill_u64(d, reinterpret_cast<uint64_t*>(t->rep), 2 * q * 32, 0) != hipSuccess)
        rc = CNMF_EHIP;
    if (!rc) rc = rsi_forward(t);
    // outer loop with checkpoints every ckpt iterations
    if (!rc && (hipMemcpyAsync(t->Gc[0], G0, (size_t)n * p * 4, hipMemcpyDeviceToDevice, d.stream) != hipSuccess ||
                hipMemcpyAsync(t->Fc[0], F0, (size_t)p * m * 4, hipMemcpyDeviceToDevice, d.stream) != hipSuccess ||
                hipMemcpyAsync(G_out, G0, (size_t)n * p * 4, hipMemcpyDeviceToDevice, d.stream) != hipSuccess ||
                hipMemcpyAsync(F_out, F0, (size_t)p * m * 4, hipMemcpyDeviceToDevice, d.stream) != hipSuccess))
        rc = CNMF_EHIP;
    for (int s = 0; !rc && s * ckpt < T; ++s) {
        const int cnt = std::min(ckpt, T - s * ckpt);
        rc = solve_span(t, G_out, F_out, s * ckpt, cnt, false);
        if (!rc && s + 1 < nck &&
            (hipMemcpyAsync(t->Gc[s + 1], G_out, (size_t)n * p * 4, hipMemcpyDeviceToDevice, d.stream) != hipSuccess ||
             hipMemcpyAsync(t->Fc[s + 1], F_out, (size_t)p * m * 4, hipMemcpyDeviceToDevice, d.stream) != hipSuccess))
            rc = CNMF_EHIP;
    }
    if (rc) {
        cnmf_tape_destroy(t);
        return rc;
    }
    *tape_out = t;
    return CNMF_OK;
}

int cnmf_adj_backward(cnmf_tape* t, const float* dG, const float* dF, float* dX, int64_t lddx,
                      float* dG0, float* dF0) {
    if (!t || bad_ptr(dG) || bad_ptr(dF) || bad_ptr(dX) || lddx < t->m) return CNMF_EINVAL;
    cnmf_ctx* c = t->c;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    const Dev& d = c->dev;
    const int64_t n = t->n, m = t->m;
    const int p = t->p, l = t->l, T = t->T, ck = t->ck;
    {   // the thin-QR adjoint is the derivative of Algorithm 2's bases only
        // when the rank rule replaced no column (a replaced column is a
        // discontinuity of the basis in X): refuse before any work
        std::vector<int32_t> flags((size_t)4 * t->q * 32);
        CK(hipMemcpyAsync(flags.data(), t->rep, flags.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, d.stream));
        CK(hipStreamSynchronize(d.stream));
        for (const int32_t f : flags)
            if (f) return CNMF_ENODERIV;
    }
    CK(copy2d(d, n, p, dG, p, t->Gb, p));
    CK(copy2d(d, p, m, dF, m, t->Fb, m));
    CK(fillf(d, (int64_t)n * l, 0.f, t->XRb));
    CK(fillf(d, (int64_t)l * m, 0.f, t->XLb));
    CK(fillf(d, (int64_t)n * l, 0.f, t->QLb));
    CK(fillf(d, (int64_t)m * l, 0.f, t->QRb));
    const int nseg = (T + ck - 1) / ck;
    for (int s = nseg - 1; s >= 0; --s) {
        const int t0 = s * ck, cnt = std::min(ck, T - t0);
        // recompute the segment from its checkpoint, keeping every iterate
        CK(hipMemcpyAsync(t->Tn, t->Gc[s], (size_t)n * p * 4, hipMemcpyDeviceToDevice, d.stream));
        CK(hipMemcpyAsync(t->Tm, t->Fc[s], (size_t)p * m * 4, hipMemcpyDeviceToDevice, d.stream));
        int rc = solve_span(t, t->Tn, t->Tm, t0, cnt, true);
        if (rc) return rc;
        // top eigenvectors of every W of the segment
        if (t->p <= 16)
            hipLaunchKernelGGL(k_eigvec<16>, dim3(2 * cnt), dim3(64), 0, d.stream, t->p, t->Wh, t->Lh, t->Vh);
        else
            hipLaunchKernelGGL(k_eigvec<32>, dim3(2 * cnt), dim3(64), 0, d.stream, t->p, t->Wh, t->Lh, t->Vh);
        CK(hipGetLastError());
        for (int j = cnt - 1; j >= 0; --j) {
            const float* Gcur = t->Gh + (size_t)j * n * p;
            const float* Gprev = j > 0 ? t->Gh + (size_t)(j - 1) * n * p : t->Gc[s];
            const float* Fprev = j > 0 ? t->Fh + (size_t)(j - 1) * p * m : t->Fc[s];
            rc = outer_adj(t, j, Gprev, Fprev, Gcur);
            if (rc) return rc;
        }
    }
    if (dG0) CK(copy2d(d, n, p, t->Gb, p, dG0, p));
    if (dF0) CK(copy2d(d, p, m, t->Fb, m, dF0, m));
    const int rc = rsi_adj(t);
    if (rc) return rc;
    const int r = 2 * (2 * t->q + 1) * l;
    dim3 grid(nb(m, 64), nb(n, 64));
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(kThreads), 0, d.stream, n, m, r, t->U, t->V, dX, lddx);
    return from_hip(hipGetLastError());
}

int cnmf_tape_destroy(cnmf_tape* t) {
    if (!t) return CNMF_OK;
    if (t->c) {
        (void)hipSetDevice(t->c->dev.device);
        (void)hipStreamSynchronize(t->c->dev.stream);
    }
    if (t->mem) (void)hipFree(t->mem);
    delete t;
    return CNMF_OK;
}

int cnmf_tape_bytes(const cnmf_tape* t, uint64_t* bytes) {
    if (!t || !bytes) return CNMF_EINVAL;
    *bytes = t->bytes;
    return CNMF_OK;
}

}  // extern "C"
