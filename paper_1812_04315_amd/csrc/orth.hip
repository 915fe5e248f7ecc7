// Orthonormal bases for randomized subspace iteration (Sec. 3, Algorithm 2:
// "QR decomposition", "orthonormal bases" of each sketch and half-step).
//
// CholeskyQR2 on an N x l FP32 panel (l <= 32):
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
#include "internal.hpp"

namespace cnmf {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxW = 64;       // augmented width 2l
constexpr int kRowsPerTile = 32;

// Partial Gram of [Y | P] over a slice of rows, FP64.  Output: upper triangle
// (a <= b) packed as a*w + b into part[blk][w*w].
__global__ __launch_bounds__(kThreads) void k_gram(int64_t N, int l, const float* __restrict__ Y,
                                                   const float* __restrict__ P, int64_t p_rs,
                                                   int64_t p_cs, int w, int64_t rows_per_blk,
                                                   double* __restrict__ part) {
    __shared__ double tile[kRowsPerTile][kMaxW + 1];
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r_end = min(N, r_begin + rows_per_blk);
    const int npairs = w * (w + 1) / 2;
    constexpr int kMaxPairs = (kMaxW * (kMaxW + 1) / 2 + kThreads - 1) / kThreads;  // 9
    double acc[kMaxPairs];
    int pa[kMaxPairs], pb[kMaxPairs];
#pragma unroll
    for (int s = 0; s < kMaxPairs; ++s) {
        acc[s] = 0.0;
        int e = threadIdx.x + s * kThreads;
        int a = 0, b = 0;
        if (e < npairs) {
            // e -> (a, b), a <= b, row-major over the upper triangle
            int rem = e;
            a = 0;
            while (rem >= w - a) { rem -= w - a; ++a; }
            b = a + rem;
        }
        pa[s] = a;
        pb[s] = (e < npairs) ? b : -1;
    }
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kRowsPerTile) {
        __syncthreads();
        for (int e = threadIdx.x; e < kRowsPerTile * w; e += kThreads) {
            const int rr = e / w, c = e - rr * w;
            const int64_t r = r0 + rr;
            double v = 0.0;
            if (r < r_end) v = (c < l) ? (double)Y[r * l + c] : (double)P[r * p_rs + (c - l) * p_cs];
            tile[rr][c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kMaxPairs; ++s) {
            if (pb[s] >= 0) {
                double t = acc[s];
                for (int rr = 0; rr < kRowsPerTile; ++rr) t = fma(tile[rr][pa[s]], tile[rr][pb[s]], t);
                acc[s] = t;
            }
        }
    }
#pragma unroll
    for (int s = 0; s < kMaxPairs; ++s)
        if (pb[s] >= 0) part[(int64_t)blockIdx.x * w * w + pa[s] * w + pb[s]] = acc[s];
}

// Cholesky with the rank rule and the inverse of R, one workgroup.
//   ws layout: Rinv[32*32] doubles, then sel[32] as doubles (0/1).
__global__ __launch_bounds__(kThreads) void k_chol(int l, int w, int nblk,
                                                   const double* __restrict__ part, double tau2,
                                                   int allow_swap, double* __restrict__ out,
                                                   int32_t* __restrict__ replaced, Control* ctl) {
    __shared__ double M[kMaxW][kMaxW + 1];
    __shared__ double R[32][33];
    __shared__ double ref[kMaxW];
    __shared__ int sel[32];
    __shared__ double s_thr;
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    for (int e = tid; e < w * w; e += kThreads) {
        const int a = e / w, b = e - a * w;
        double v = 0.0;
        if (a <= b) {
            for (int k = 0; k < nblk; ++k) v += part[(int64_t)k * w * w + a * w + b];
            M[a][b] = v;
            M[b][a] = v;
        }
    }
    __syncthreads();
    if (tid < w) ref[tid] = M[tid][tid];
    if (tid < 32) sel[tid] = 0;
    for (int e = tid; e < 32 * 33; e += kThreads) R[e / 33][e % 33] = 0.0;
    __syncthreads();
    if (tid == 0) {
        double mx = 0.0;
        int bad = 0;
        for (int i = 0; i < l; ++i) {
            if (!isfinite(ref[i])) bad = 1;
            mx = fmax(mx, ref[i]);
        }
        for (int i = l; i < w; ++i) if (!isfinite(ref[i])) bad = 1;
        if (bad) raise_status(ctl, CNMF_ST_NONFINITE);
        s_thr = tau2 * mx;
    }
    __syncthreads();
    for (int j = 0; j < l; ++j) {
        if (tid == 0) {
            const double d = M[j][j];
            int f = 0;
            if (allow_swap) {
                if (!(d > s_thr)) f = 1;
            } else if (!(d > tau2 * ref[j])) {
                f = 2;
            }
            s_flag = f;
        }
        __syncthreads();
        if (s_flag == 1) {
            // swap rows j and l + j, then columns j and l + j
            for (int c = tid; c < w; c += kThreads) {
                double t = M[j][c]; M[j][c] = M[l + j][c]; M[l + j][c] = t;
            }
            __syncthreads();
            for (int r = tid; r < w; r += kThreads) {
                double t = M[r][j]; M[r][j] = M[r][l + j]; M[r][l + j] = t;
            }
            __syncthreads();
            if (tid == 0) {
                sel[j] = 1;
                if (!(M[j][j] > tau2 * ref[l + j])) s_flag = 2;
            }
            __syncthreads();
        }
        if (s_flag == 2) {
            if (tid == 0) {
                raise_status(ctl, CNMF_ST_BREAKDOWN);
                M[j][j] = 1.0;   // keep going; the status word marks the result invalid
                for (int c = j + 1; c < w; ++c) { M[j][c] = 0.0; M[c][j] = 0.0; }
            }
            __syncthreads();
        }
        const double rjj = sqrt(M[j][j]);
        // row j of the factor over all remaining columns (pool included)
        __shared__ double rowj[kMaxW];
        for (int c = tid; c < w; c += kThreads) rowj[c] = (c > j) ? M[j][c] / rjj : 0.0;
        if (tid == 0) rowj[j] = rjj;
        __syncthreads();
        if (tid < l) R[j][tid] = (tid >= j) ? rowj[tid] : 0.0;
        const int t = w - j - 1;
        for (int e = tid; e < t * t; e += kThreads) {
            const int a = j + 1 + e / t, b = j + 1 + e % t;
            M[a][b] -= rowj[a] * rowj[b];
        }
        __syncthreads();
    }
    // Rinv: thread c computes column c by back substitution.
    __shared__ double Ri[32][33];
    if (tid < l) {
        const int c = tid;
        for (int i = 0; i < l; ++i) Ri[i][c] = 0.0;
        Ri[c][c] = 1.0 / R[c][c];
        for (int i = c - 1; i >= 0; --i) {
            double s = 0.0;
            for (int t2 = i + 1; t2 <= c; ++t2) s = fma(R[i][t2], Ri[t2][c], s);
            Ri[i][c] = -s / R[i][i];
        }
    }
    __syncthreads();
    for (int e = tid; e < 32 * 32; e += kThreads) {
        const int i = e / 32, c = e % 32;
        out[e] = (i < l && c < l) ? Ri[i][c] : 0.0;
    }
    if (tid < 32) {
        out[32 * 32 + tid] = (tid < l) ? (double)sel[tid] : 0.0;
        if (replaced && tid < l) replaced[tid] = sel[tid];
    }
}

// Q[r][:] = Y^[r][:] * Rinv, FP64 arithmetic, one row per thread.
__global__ __launch_bounds__(kThreads) void k_apply(int64_t N, int l, const float* __restrict__ Y,
                                                    const float* __restrict__ P, int64_t p_rs,
                                                    int64_t p_cs, const double* __restrict__ rs,
                                                    float* __restrict__ Q) {
    __shared__ double Ri[32][32];
    __shared__ int sel[32];
    for (int e = threadIdx.x; e < 32 * 32; e += kThreads) Ri[e / 32][e % 32] = rs[e];
    if (threadIdx.x < 32) sel[threadIdx.x] = rs[32 * 32 + threadIdx.x] != 0.0;
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= N) return;
    double y[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        if (i < l) y[i] = sel[i] ? (double)P[r * p_rs + i * p_cs] : (double)Y[r * l + i];
        else y[i] = 0.0;
    }
    for (int c = 0; c < l; ++c) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 32; ++i)
            if (i <= c) s = fma(y[i], Ri[i][c], s);
        Q[r * l + c] = (float)s;
    }
}

int64_t gram_blocks(const Dev& d, int64_t N) {
    int64_t b = (N + 255) / 256;
    if (b > d.num_cus) b = d.num_cus;
    return b < 1 ? 1 : b;
}

}  // namespace

size_t orth_workspace_doubles(const Dev& d, int64_t N, int l) {
    const int w = 2 * l;
    return (size_t)gram_blocks(d, N) * w * w + 2 * (32 * 32 + 32);
}

hipError_t orth(const Dev& d, int64_t N, int l, const float* Y, const float* pool,
                bool pool_trans, double tau2, float* Q, int32_t* replaced, double* ws,
                Control* ctl) {
    if (N <= 0 || l <= 0) return hipSuccess;
    const int64_t nb = gram_blocks(d, N);
    const int64_t rpb = (N + nb - 1) / nb;
    const int64_t p_rs = pool_trans ? 1 : l;
    const int64_t p_cs = pool_trans ? N : 1;
    double* part = ws;
    double* rs = ws + (size_t)nb * (2 * l) * (2 * l);
    // pass 1: augmented Gram, Cholesky with swaps, Q1 = Y^ R^-1 (into Q)
    hipLaunchKernelGGL(k_gram, dim3((unsigned)nb), dim3(kThreads), 0, d.stream, N, l, Y, pool,
                       p_rs, p_cs, 2 * l, rpb, part);
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(kThreads), 0, d.stream, l, 2 * l, (int)nb, part,
                       tau2, 1, rs, replaced, ctl);
    hipLaunchKernelGGL(k_apply, dim3((unsigned)((N + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, d.stream, N, l, Y, pool, p_rs, p_cs, rs, Q);
    // pass 2 on Q1 (no swaps), in place
    hipLaunchKernelGGL(k_gram, dim3((unsigned)nb), dim3(kThreads), 0, d.stream, N, l, Q, Q,
                       (int64_t)l, (int64_t)1, l, rpb, part);
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(kThreads), 0, d.stream, l, l, (int)nb, part, tau2,
                       0, rs, (int32_t*)nullptr, ctl);
    hipLaunchKernelGGL(k_apply, dim3((unsigned)((N + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, d.stream, N, l, Q, Q, (int64_t)l, (int64_t)1, rs, Q);
    return hipGetLastError();
}

}  // namespace cnmf
