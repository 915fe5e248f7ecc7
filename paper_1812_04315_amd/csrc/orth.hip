// Orthonormal bases for randomized subspace iteration (Sec. 3, Algorithm 2:
// "QR decomposition", "orthonormal bases" of each sketch and half-step).
//
// CholeskyQR2 on an N x l FP32 panel (l <= 32), one persistent launch:
//   pass 1: W = [Y P]^T [Y P] in FP64 (P = replacement pool), right-looking
//           Cholesky of W with the numerical-rank rule, Q1 = Y^ R^-1 where Y^
//           is Y with deficient columns swapped for pool columns;
//   pass 2: W = Q1^T Q1, Cholesky, Q = Q1 R2^-1.
// The FP64 Gram of FP32 data has exact products, so pass 1 already gives
// orthogonality near FP32 rounding for condition numbers far beyond what the
// rank rule admits; pass 2 removes what is left.
//
// Rank rule: at Cholesky step j the Schur-complement pivot d_j is the squared
// residual of column j after projection onto columns < j.  d_j <=
// tau2 * max_i ||y_i||^2 marks column j deficient; it is swapped (symmetric
// row/column permutation of the augmented Gram, whose pool part has been
// eliminated alongside) for pool column j.  A swapped-in column whose pivot
// is <= tau2 * ||pool_j||^2 is a breakdown.
//
// Each workgroup owns a contiguous slice of rows.  Gram partials are summed
// across the grid through tagged 64-bit words (the tag in the upper half,
// half of an FP64 value in the lower): every workgroup publishes its
// partial, reduces a share of the entries over all partials and publishes
// the sums, then reads every sum; each workgroup then factors the (tiny)
// Gram itself.  No fences and no second launch are needed.
#include "internal.hpp"

namespace cnmf {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxW = 64;        // augmented width 2 l
constexpr int kMaxPairs = kMaxW * (kMaxW + 1) / 2;   // 2080
constexpr int kPairsPerThread = (kMaxPairs + kThreads - 1) / kThreads;   // 9
constexpr int kTile = 32;

__device__ __forceinline__ void xstore(uint64_t* p, unsigned tag, double v) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    __hip_atomic_store(p, ((uint64_t)tag << 32) | (bits >> 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, ((uint64_t)tag << 32) | (bits & 0xffffffffu), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true and the value when both words carry `tag`.
__device__ __forceinline__ bool xload(const uint64_t* p, unsigned tag, double* v) {
    const uint64_t w0 = __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t w1 = __hip_atomic_load(const_cast<uint64_t*>(p + 1), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    if ((unsigned)(w0 >> 32) != tag || (unsigned)(w1 >> 32) != tag) return false;
    *v = __longlong_as_double((long long)((w0 << 32) | (w1 & 0xffffffffu)));
    return true;
}

__device__ __forceinline__ void pair_of(int e, int w, int* a, int* b) {
    int rem = e, r = 0;
    while (rem >= w - r) { rem -= w - r; ++r; }
    *a = r;
    *b = r + rem;
}

struct Shared {
    double M[kMaxW][kMaxW + 1];
    double tile[kTile][kMaxW + 1];
    double Ri[32][33];
    double rvec[kMaxW];
    double ref[kMaxW];
    int sel[32];
    int flag;
    int timeout;
};

}  // namespace

struct OrthArgs {
    int64_t N;
    int l;
    const float* Y;
    const float* P;
    int64_t p_rs, p_cs;
    double tau2;
    float* Q;           // N x l
    float* QT;          // optional l x N copy, row pitch ldqt
    int64_t ldqt;
    int32_t* replaced;  // optional l flags
    uint64_t* part;     // [nblk][kMaxPairs][2]
    uint64_t* red;      // [kMaxPairs][2]
    unsigned seq;
    Control* ctl;
};

namespace {

// Gram partial over this workgroup's rows: pairs (a <= b) of the w columns of
// [A | P] (w = l: only A).  A element (r, c) at A[r * l + c].
__device__ void gram_partial(const OrthArgs& g, Shared& sh, const float* A, int w, int64_t r0,
                             int64_t r1, double (&acc)[kPairsPerThread], int (&pa)[kPairsPerThread],
                             int (&pb)[kPairsPerThread]) {
    const int npairs = w * (w + 1) / 2;
#pragma unroll
    for (int s = 0; s < kPairsPerThread; ++s) {
        acc[s] = 0.0;
        const int e = threadIdx.x + s * kThreads;
        int a = 0, b = -1;
        if (e < npairs) pair_of(e, w, &a, &b);
        pa[s] = a;
        pb[s] = b;
    }
    const int l = g.l;
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        __syncthreads();
        for (int e = threadIdx.x; e < kTile * w; e += kThreads) {
            const int rr = e / w, c = e - rr * w;
            const int64_t r = t0 + rr;
            double v = 0.0;
            if (r < r1) v = (c < l) ? (double)A[r * l + c] : (double)g.P[r * g.p_rs + (c - l) * g.p_cs];
            sh.tile[rr][c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kPairsPerThread; ++s) {
            if (pb[s] >= 0) {
                double t = acc[s];
                for (int rr = 0; rr < kTile; ++rr) t = fma(sh.tile[rr][pa[s]], sh.tile[rr][pb[s]], t);
                acc[s] = t;
            }
        }
    }
}

// Sum of the partial Grams over the grid -> sh.M (full symmetric, w x w).
// Returns false on a stalled exchange.
__device__ bool gram_exchange(const OrthArgs& g, Shared& sh, int w, unsigned tag_part,
                              unsigned tag_red, const double (&acc)[kPairsPerThread],
                              const int (&pa)[kPairsPerThread], const int (&pb)[kPairsPerThread]) {
    const int npairs = w * (w + 1) / 2;
    const unsigned nblk = gridDim.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // 1. publish this workgroup's partial
#pragma unroll
    for (int s = 0; s < kPairsPerThread; ++s) {
        const int e = threadIdx.x + s * kThreads;
        if (e < npairs) xstore(g.part + ((size_t)blockIdx.x * kMaxPairs + e) * 2, tag_part, acc[s]);
    }
    // 2. reduce a share of the entries over all partials, one wave per entry
    if (threadIdx.x == 0) sh.timeout = 0;
    __syncthreads();
    for (int e = blockIdx.x + nblk * wave; e < npairs; e += nblk * 4) {
        unsigned spins = 0;
        double t;
        for (;;) {
            int ok = 1;
            t = 0.0;
            for (unsigned i = lane; i < nblk; i += 64) {
                double v;
                if (xload(g.part + ((size_t)i * kMaxPairs + e) * 2, tag_part, &v)) t += v;
                else ok = 0;
            }
            if (__all(ok)) break;
            __builtin_amdgcn_s_sleep(1);
            int to = 0;
            if (((++spins) & 255u) == 0u)
                to = spins >= (kSpinLimit >> 4) || (atomic_status_load(&g.ctl->status) & CNMF_ST_TIMEOUT);
            if (__any(to)) {
                if (lane == 0) { raise_status(g.ctl, CNMF_ST_TIMEOUT); sh.timeout = 1; }
                break;
            }
        }
        t = wave_sum(t);
        if (lane == 0) xstore(g.red + (size_t)e * 2, tag_red, t);
    }
    __syncthreads();
    if (sh.timeout) return false;
    // 3. read every sum
    unsigned spins = 0;
    for (;;) {
        int ok = 1;
        for (int e = threadIdx.x; e < npairs; e += kThreads) {
            double v;
            if (xload(g.red + (size_t)e * 2, tag_red, &v)) {
                int a, b;
                pair_of(e, w, &a, &b);
                sh.M[a][b] = v;
                sh.M[b][a] = v;
            } else {
                ok = 0;
            }
        }
        if (__syncthreads_and(ok)) break;
        __builtin_amdgcn_s_sleep(1);
        ++spins;
        int to = 0;
        if (threadIdx.x == 0 && (spins & 255u) == 0u)
            to = spins >= (kSpinLimit >> 4) || (atomic_status_load(&g.ctl->status) & CNMF_ST_TIMEOUT);
        if (__syncthreads_or(to)) {
            if (threadIdx.x == 0) raise_status(g.ctl, CNMF_ST_TIMEOUT);
            return false;
        }
    }
    return true;
}

// Right-looking Cholesky of sh.M (w x w) over the first l pivots by one
// wavefront (lane i owns row i), with the rank rule when allow_swap; R^-1 of
// the leading l x l factor into sh.Ri, swap flags into sh.sel.
__device__ void cholesky_wave(const OrthArgs& g, Shared& sh, int w, bool allow_swap) {
    const int lane = threadIdx.x;   // wave 0 only
    const int l = g.l;
    if (lane < w) sh.ref[lane] = sh.M[lane][lane];
    if (lane < 32) sh.sel[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    double mx = 0.0;
    int bad = 0;
    for (int i = 0; i < w; ++i) {
        const double v = sh.ref[i];
        if (!isfinite(v)) bad = 1;
        if (i < l) mx = fmax(mx, v);
    }
    if (bad && lane == 0) raise_status(g.ctl, CNMF_ST_NONFINITE);
    const double thr = g.tau2 * mx;
    double rrow[32];   // R[j][lane] for j < l (row j of R lives in lane's column)
#pragma unroll
    for (int j = 0; j < 32; ++j) rrow[j] = 0.0;
    for (int j = 0; j < l; ++j) {
        double d = sh.M[j][j];
        int flag = 0;
        if (allow_swap) {
            if (!(d > thr)) flag = 1;
        } else if (!(d > g.tau2 * sh.ref[j])) {
            flag = 2;
        }
        if (flag == 1) {
            // swap rows / columns j and l + j of the augmented matrix
            if (lane < w) {
                const double t = sh.M[j][lane];
                sh.M[j][lane] = sh.M[l + j][lane];
                sh.M[l + j][lane] = t;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < w) {
                const double t = sh.M[lane][j];
                sh.M[lane][j] = sh.M[lane][l + j];
                sh.M[lane][l + j] = t;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) sh.sel[j] = 1;
            d = sh.M[j][j];
            if (!(d > g.tau2 * sh.ref[l + j])) flag = 2;
        }
        if (flag == 2) {
            if (lane == 0) raise_status(g.ctl, CNMF_ST_BREAKDOWN);
            d = 1.0;
            if (lane > j && lane < w) {
                sh.M[j][lane] = 0.0;
                sh.M[lane][j] = 0.0;
            }
            __builtin_amdgcn_wave_barrier();
        }
        const double rjj = sqrt(d);
        // row j of the factor: r_i = M[j][i] / rjj for i > j, rjj at i = j
        const double ri = (lane > j && lane < w) ? sh.M[j][lane] / rjj : (lane == j ? rjj : 0.0);
        if (lane < w) sh.rvec[lane] = ri;
#pragma unroll
        for (int jj = 0; jj < 32; ++jj)
            if (jj == j) rrow[jj] = ri;
        __builtin_amdgcn_wave_barrier();
        if (lane > j && lane < w)
            for (int b = j + 1; b < w; ++b) sh.M[lane][b] -= ri * sh.rvec[b];
        __builtin_amdgcn_wave_barrier();
    }
    // R (l x l) to LDS: R[j][lane] = rrow[j]
    if (lane < l) {
#pragma unroll
        for (int j = 0; j < 32; ++j)
            if (j < l) sh.M[j][lane] = rrow[j];
    }
    __builtin_amdgcn_wave_barrier();
    // R^-1 by back substitution, lane c owns column c
    if (lane < l) {
        const int c = lane;
        for (int i = 0; i < l; ++i) sh.Ri[i][c] = 0.0;
        sh.Ri[c][c] = 1.0 / sh.M[c][c];
        for (int i = c - 1; i >= 0; --i) {
            double s = 0.0;
            for (int t = i + 1; t <= c; ++t) s = fma(sh.M[i][t], sh.Ri[t][c], s);
            sh.Ri[i][c] = -s / sh.M[i][i];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Q[r][:] = Ysrc^[r][:] * Ri over this workgroup's rows (FP64 arithmetic).
__device__ void apply_rows(const OrthArgs& g, Shared& sh, const float* Ysrc, bool use_pool,
                           int64_t r0, int64_t r1, float* Qdst, float* QT) {
    const int l = g.l;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kThreads) {
        double y[32];
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            if (i < l) y[i] = (use_pool && sh.sel[i]) ? (double)g.P[r * g.p_rs + i * g.p_cs]
                                                      : (double)Ysrc[r * l + i];
            else y[i] = 0.0;
        }
        for (int c = 0; c < l; ++c) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < 32; ++i)
                if (i <= c) s = fma(y[i], sh.Ri[i][c], s);
            Qdst[r * l + c] = (float)s;
            if (QT) QT[(int64_t)c * g.ldqt + r] = (float)s;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_orth(OrthArgs g) {
    __shared__ Shared sh;
    const unsigned nblk = gridDim.x;
    const int64_t rpw = (g.N + nblk - 1) / nblk;
    const int64_t r0 = (int64_t)blockIdx.x * rpw;
    const int64_t r1 = min(g.N, r0 + rpw);
    const int l = g.l;
    double acc[kPairsPerThread];
    int pa[kPairsPerThread], pb[kPairsPerThread];

    // pass 1: augmented Gram, Cholesky with swaps, Q1 = Y^ R^-1 (into Q)
    gram_partial(g, sh, g.Y, 2 * l, r0, r1, acc, pa, pb);
    if (!gram_exchange(g, sh, 2 * l, (g.seq << 10) | 1u, (g.seq << 10) | 2u, acc, pa, pb)) return;
    if (threadIdx.x < 64) cholesky_wave(g, sh, 2 * l, true);
    __syncthreads();
    if (blockIdx.x == 0 && g.replaced && threadIdx.x < l) g.replaced[threadIdx.x] = sh.sel[threadIdx.x];
    apply_rows(g, sh, g.Y, true, r0, r1, g.Q, nullptr);
    __threadfence_block();
    __syncthreads();

    // pass 2 on Q1 (no swaps), in place
    gram_partial(g, sh, g.Q, l, r0, r1, acc, pa, pb);
    if (!gram_exchange(g, sh, l, (g.seq << 10) | 3u, (g.seq << 10) | 4u, acc, pa, pb)) return;
    if (threadIdx.x < 64) cholesky_wave(g, sh, l, false);
    __syncthreads();
    apply_rows(g, sh, g.Q, false, r0, r1, g.Q, g.QT);
}

unsigned orth_blocks(const Dev& d, int64_t N) {
    int64_t b = (N + 255) / 256;
    if (b > d.num_cus) b = d.num_cus;
    if (b > 256) b = 256;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

size_t orth_exchange_words() { return (size_t)257 * kMaxPairs * 2; }

hipError_t orth(const Dev& d, int64_t N, int l, const float* Y, const float* pool,
                bool pool_trans, double tau2, float* Q, float* QT, int64_t ldqt,
                int32_t* replaced, uint64_t* xch, unsigned seq, Control* ctl) {
    if (N <= 0 || l <= 0) return hipSuccess;
    if (l > 32 || seq >= (1u << 22)) return hipErrorInvalidValue;
    OrthArgs g;
    g.N = N;
    g.l = l;
    g.Y = Y;
    g.P = pool;
    g.p_rs = pool_trans ? 1 : l;
    g.p_cs = pool_trans ? N : 1;
    g.tau2 = tau2;
    g.Q = Q;
    g.QT = QT;
    g.ldqt = ldqt;
    g.replaced = replaced;
    g.part = xch + (size_t)kMaxPairs * 2;
    g.red = xch;
    g.seq = seq;
    g.ctl = ctl;
    hipLaunchKernelGGL(k_orth, dim3(orth_blocks(d, N)), dim3(kThreads), 0, d.stream, g);
    return hipGetLastError();
}

}  // namespace cnmf
