// Small-matrix and measurement kernels:
//   * Lipschitz constant of the inner loop's gradient map (Sec. 2: a single
//     gradient step per inner iteration; step 1/L with L = lambda_max(W)),
//     in FP64 by Householder tridiagonalisation and Sturm bisection;
//   * gradient-bound initialisation and device clock stamps;
//   * relative reconstruction error (Sec. 4, Eq. (4)).
#include "internal.hpp"

namespace cnmf {

namespace {

// One wavefront.  A = (W + W^T) / 2 in FP64, reduced to tridiagonal form by
// Householder reflections H = I - 2 v v^T (lane i owns row i); the largest
// eigenvalue of the tridiagonal matrix is then bracketed between max_i d_i
// and its Gershgorin bound and narrowed by 64-way Sturm multisection.
__global__ __launch_bounds__(64) void k_lipschitz(int p, const float* __restrict__ W,
                                                  double* __restrict__ out, Control* ctl) {
    __shared__ double A[32][33];
    __shared__ double v[32], wv[32];
    __shared__ double dg[32], eo[32];
    const int lane = threadIdx.x;
    for (int e = lane; e < p * p; e += 64) {
        const int i = e / p, j = e % p;
        A[i][j] = 0.5 * ((double)W[i * p + j] + (double)W[j * p + i]);
    }
    __syncthreads();
    for (int k = 0; k + 2 < p; ++k) {
        const int i = lane;
        const bool in = (i > k) && (i < p);
        const double xi = in ? A[i][k] : 0.0;
        const double sigma = wave_sum(xi * xi);
        const double x0 = A[k + 1][k];
        if (sigma == 0.0) {
            if (lane == 0) { dg[k] = A[k][k]; eo[k] = 0.0; }
            __syncthreads();
            continue;
        }
        const double alpha = -copysign(sqrt(sigma), x0);
        const double v0 = x0 - alpha;
        const double vn = sqrt(sigma - x0 * x0 + v0 * v0);
        if (in) v[i] = ((i == k + 1) ? v0 : xi) / vn;
        __syncthreads();
        double ui = 0.0;
        if (in)
            for (int j = k + 1; j < p; ++j) ui = fma(A[i][j], v[j], ui);
        const double c = wave_sum(in ? v[i] * ui : 0.0);
        if (in) wv[i] = 2.0 * ui - 2.0 * c * v[i];
        __syncthreads();
        if (in)
            for (int j = k + 1; j < p; ++j) A[i][j] -= v[i] * wv[j] + wv[i] * v[j];
        if (lane == 0) { dg[k] = A[k][k]; eo[k] = alpha; }
        __syncthreads();
    }
    if (lane == 0) {
        if (p >= 2) {
            dg[p - 2] = A[p - 2][p - 2];
            eo[p - 2] = A[p - 1][p - 2];
        }
        dg[p - 1] = A[p - 1][p - 1];
    }
    __syncthreads();
    // Bracket [lo, hi] around lambda_max.
    double lo = -INFINITY, hi = -INFINITY, emax = 0.0;
    bool bad = false;
    for (int i = 0; i < p; ++i) {
        const double el = (i > 0) ? fabs(eo[i - 1]) : 0.0;
        const double er = (i + 1 < p) ? fabs(eo[i]) : 0.0;
        lo = fmax(lo, dg[i]);
        hi = fmax(hi, dg[i] + el + er);
        emax = fmax(emax, er);
        if (!isfinite(dg[i]) || !isfinite(er)) bad = true;
    }
    if (bad) {
        if (lane == 0) { out[0] = NAN; raise_status(ctl, CNMF_ST_NONFINITE); }
        return;
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax * emax);
    for (int round = 0; round < 16 && hi > lo; ++round) {
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        // Sturm count: eigenvalues below x
        int cnt = 0;
        double q = dg[0] - x;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
        for (int i = 1; i < p; ++i) {
            q = (dg[i] - x) - eo[i - 1] * eo[i - 1] / q;
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += q < 0.0;
        }
        const bool above = (cnt == p);   // lambda_max < x
        const unsigned long long mask = __ballot(above);
        double nlo = lo, nhi = hi;
        if (mask) {
            const int first = __ffsll((long long)mask) - 1;
            nhi = __shfl(x, first, 64);
            if (first > 0) nlo = __shfl(x, first - 1, 64);
        } else {
            nlo = __shfl(x, 63, 64);
        }
        if (!(nhi - nlo < hi - lo)) break;
        lo = nlo;
        hi = nhi;
        if (hi - lo <= 4.0 * 2.220446049250313e-16 * fabs(hi)) break;
    }
    if (lane == 0) out[0] = hi;
}

__global__ void k_tol_init(Control* ctl, double ratio) {
    if (threadIdx.x == 0) {
        const double t = ratio * sqrt(ctl->pg2[0] + ctl->pg2[1]);
        ctl->tol[0] = t;
        ctl->tol[1] = t;
        if (!isfinite(t)) raise_status(ctl, CNMF_ST_NONFINITE);
    }
}

__global__ void k_fill_u64(uint64_t* p, int64_t count, uint64_t value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

__global__ void k_tick(unsigned long long* t) {
    if (threadIdx.x == 0) t[0] = wall_clock64();
}

// Residual ||X - G F||^2 (FP64 accumulation) for snapshot blockIdx.y over
// the row slice of workgroup blockIdx.x; ||X||^2 in slot `count`.
constexpr int kRowsR = 8;
__global__ __launch_bounds__(256) void k_rre(int64_t n, int64_t m, const float* __restrict__ X,
                                             int64_t ldx, int p, const float* __restrict__ G,
                                             int64_t sG, const float* __restrict__ F, int64_t sF,
                                             int count, int64_t rows_per_blk,
                                             double* __restrict__ part) {
    __shared__ float g[kRowsR][32];
    __shared__ double red[4];
    const int snap = blockIdx.y;
    const bool xnorm = (snap == count);
    const float* Gs = G + (xnorm ? 0 : (int64_t)snap * sG);
    const float* Fs = F + (xnorm ? 0 : (int64_t)snap * sF);
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r_end = min(n, r_begin + rows_per_blk);
    double acc = 0.0;
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kRowsR) {
        __syncthreads();
        if (!xnorm)
            for (int e = threadIdx.x; e < kRowsR * p; e += 256) {
                const int rr = e / p, c = e % p;
                g[rr][c] = (r0 + rr < r_end) ? Gs[(r0 + rr) * p + c] : 0.f;
            }
        __syncthreads();
        for (int64_t j = threadIdx.x; j < m; j += 256) {
            float f[32];
            if (!xnorm)
                for (int c = 0; c < p; ++c) f[c] = Fs[(int64_t)c * m + j];
            for (int rr = 0; rr < kRowsR; ++rr) {
                const int64_t r = r0 + rr;
                if (r >= r_end) break;
                float s = X[r * ldx + j];
                if (!xnorm)
                    for (int c = 0; c < p; ++c) s -= g[rr][c] * f[c];
                acc = fma((double)s, (double)s, acc);
            }
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(int64_t)snap * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_rre_final(int count, int nb, const double* __restrict__ part,
                            double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double s = 0.0, x = 0.0;
    for (int b = 0; b < nb; ++b) {
        s += part[(int64_t)i * nb + b];
        x += part[(int64_t)count * nb + b];
    }
    out[i] = sqrt(s / x);
}

int64_t rre_blocks(const Dev& d, int64_t n) {
    int64_t b = (n + kRowsR * 4 - 1) / (kRowsR * 4);
    if (b > 2 * d.num_cus) b = 2 * d.num_cus;
    return b < 1 ? 1 : b;
}

}  // namespace

hipError_t lipschitz(const Dev& d, int p, const float* W, double* out, Control* ctl) {
    hipLaunchKernelGGL(k_lipschitz, dim3(1), dim3(64), 0, d.stream, p, W, out, ctl);
    return hipGetLastError();
}

hipError_t tol_init(const Dev& d, Control* ctl, double ratio) {
    hipLaunchKernelGGL(k_tol_init, dim3(1), dim3(64), 0, d.stream, ctl, ratio);
    return hipGetLastError();
}

hipError_t write_tick(const Dev& d, unsigned long long* tick) {
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, d.stream, tick);
    return hipGetLastError();
}

hipError_t fill_u64(const Dev& d, uint64_t* p, int64_t count, uint64_t value) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, d.stream, p,
                       count, value);
    return hipGetLastError();
}

size_t rre_partial_doubles(const Dev& d, int64_t n, int64_t m, int count) {
    (void)m;
    return (size_t)rre_blocks(d, n) * (count + 1);
}

hipError_t rre(const Dev& d, int64_t n, int64_t m, const float* X, int64_t ldx, int p,
               const float* G, int64_t sG, const float* F, int64_t sF, int count, double* out,
               double* partial, int64_t partial_len) {
    (void)partial_len;
    if (count <= 0) return hipSuccess;
    const int64_t nb = rre_blocks(d, n);
    const int64_t rpb = (n + nb - 1) / nb;
    hipLaunchKernelGGL(k_rre, dim3((unsigned)nb, (unsigned)(count + 1)), dim3(256), 0, d.stream,
                       n, m, X, ldx, p, G, sG, F, sF, count, rpb, partial);
    hipLaunchKernelGGL(k_rre_final, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, d.stream,
                       count, (int)nb, partial, out);
    return hipGetLastError();
}

}  // namespace cnmf
