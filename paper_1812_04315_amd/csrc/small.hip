// Measurement and bookkeeping kernels: device clock stamps, fills, and the
// relative reconstruction error of Sec. 4, Eq. (4).
#include "internal.hpp"

namespace cnmf {

namespace {

__global__ void k_fill_u64(uint64_t* p, int64_t count, uint64_t value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t value) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

__global__ void k_tick(unsigned long long* t) {
    if (threadIdx.x == 0) t[0] = wall_clock64();
}

__global__ void k_arm_deadline(Control* ctl, unsigned long long ticks) {
    if (threadIdx.x == 0) {
        ctl->deadline = wall_clock64() + ticks;
        ctl->stop = 0;
    }
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

// dst = s * src over a rows x cols block (row pitches lds, ldd; src may be
// dst).  s is the constant `scale`, or 1 / sqrt(sum of `np` partial sums)
// when `part` is given (every thread sums the partials in the same order).
__global__ void k_scale2d(int64_t rows, int64_t cols, const float* src, int64_t lds, float* dst,
                          int64_t ldd, float scale, const double* part, int np) {
    float sc = scale;
    if (part) {
        double t = 0.0;
        for (int i = 0; i < np; ++i) t += part[i];
        sc = t > 0.0 ? (float)(1.0 / sqrt(t)) : 1.f;
    }
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / cols, c = e % cols;
        dst[r * ldd + c] = sc * src[r * lds + c];
    }
}

// part[block] = sum of squares of this block's share of a rows x cols block
// (FP64, fixed order: repeatable)
__global__ __launch_bounds__(256) void k_norm2_part(int64_t rows, int64_t cols, const float* A,
                                                    int64_t lda, double* part) {
    __shared__ double red[4];
    const int64_t total = rows * cols;
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double v = A[(e / cols) * lda + e % cols];
        acc = fma(v, v, acc);
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

int64_t rre_blocks(const Dev& d, int64_t n) {
    int64_t b = (n + kRowsR * 4 - 1) / (kRowsR * 4);
    if (b > 2 * d.num_cus) b = 2 * d.num_cus;
    return b < 1 ? 1 : b;
}

}  // namespace

hipError_t write_tick(const Dev& d, unsigned long long* tick) {
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, d.stream, tick);
    return hipGetLastError();
}

hipError_t arm_deadline(const Dev& d, Control* ctl, unsigned long long ticks) {
    hipLaunchKernelGGL(k_arm_deadline, dim3(1), dim3(64), 0, d.stream, ctl, ticks);
    return hipGetLastError();
}

hipError_t scale2d(const Dev& d, int64_t rows, int64_t cols, const float* src, int64_t lds,
                   float* dst, int64_t ldd, float scale) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale2d, dim3(256), dim3(256), 0, d.stream, rows, cols, src, lds, dst, ldd,
                       scale, (const double*)nullptr, 0);
    return hipGetLastError();
}

hipError_t normalize2d(const Dev& d, int64_t rows, int64_t cols, float* A, int64_t lda,
                       double* part) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_norm2_part, dim3(kNormBlocks), dim3(256), 0, d.stream, rows, cols, A, lda,
                       part);
    hipLaunchKernelGGL(k_scale2d, dim3(256), dim3(256), 0, d.stream, rows, cols, A, lda, A, lda,
                       1.f, (const double*)part, kNormBlocks);
    return hipGetLastError();
}

hipError_t fill_u64(const Dev& d, uint64_t* p, int64_t count, uint64_t value) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, d.stream, p,
                       count, value);
    return hipGetLastError();
}

hipError_t fill_i32(const Dev& d, int32_t* p, int64_t count, int32_t value) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, d.stream, p,
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
