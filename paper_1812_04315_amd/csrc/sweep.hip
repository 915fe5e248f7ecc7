// X-sized sweeps: Y = X A (right) and Z = X^T B (left) for skinny A, B
// (k <= 32 columns).  These are the products of Algorithm 2 (X Omega_L,
// Omega_R X, X^T Q, Q X^T, X Q~, Q~ X) and of plain NeNMF's subproblem
// data X F^T and G^T X (Eqs. (2)-(3)).  They are HBM-bound: every X element
// is read once and feeds 2k flops.
//
// FP32 path: v_mfma_f32_32x32x2f32 tiles (FP32 in, FP32 accumulate).
// Non-packed FP32 VALU tops out near the HBM rate at these intensities, the
// matrix cores have twice that throughput.
//
// Split-K: the reduction dimension is cut into S slices, one slice per
// workgroup row of the grid; the 4 waves of a workgroup reduce through LDS
// and each workgroup writes one partial tile.  A second kernel sums the S
// partials in a fixed order, so results are bitwise reproducible.
#include "internal.hpp"

namespace cnmf {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ v16f mfma32(float a, float b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row of the 32x32 accumulator tile held in register r of lane l.
__device__ __forceinline__ int acc_row(int r, int lane) {
    return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// ---------------------------------------------------------------------------
// Right sweep.  Workgroup = 32 rows of X; its 4 waves take interleaved
// 32-column chunks of the workgroup's K slice.  Lane l holds row (l % 32)
// and the 16 consecutive columns starting at chunk + 16 (l / 32); element s
// feeds MFMA s, whose K index (l / 32) therefore stands for column
// chunk + 16 (l / 32) + s.  The B operand of MFMA s is A at that column
// (row of A) and output column l % 32.
// ---------------------------------------------------------------------------
template <bool A_T, bool VEC, bool DIRECT>
__global__ __launch_bounds__(kThreads) void k_sweep_right(
    int64_t R, int64_t C, const float* __restrict__ X, int64_t ldx, int k,
    const float* __restrict__ A, int64_t lda, float* __restrict__ out, int64_t ldo,
    int64_t chunks_per_split) {
    __shared__ float red[4][16][kWave];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int mr = lane & 31;
    const int kh = lane >> 5;
    const int64_t row0 = (int64_t)blockIdx.x * 32;
    const int64_t nchunks = (C + 31) / 32;
    const int64_t c_begin = (int64_t)blockIdx.y * chunks_per_split;
    const int64_t c_end = min(nchunks, c_begin + chunks_per_split);
    const int64_t xrow = row0 + mr;
    const bool rowok = xrow < R;
    const float* xr = X + (rowok ? xrow : 0) * ldx;
    const bool colok = mr < k;
    const float* ar = A_T ? A + (colok ? mr : 0) * lda : A + (colok ? mr : 0);

    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;

    for (int64_t ch = c_begin + wave; ch < c_end; ch += 4) {
        const int64_t j0 = ch * 32 + kh * 16;
        float xv[16], av[16];
        const bool full = (j0 + 16 <= C);
        if (VEC && full) {
            const v4f* p = reinterpret_cast<const v4f*>(xr + j0);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                v4f v = rowok ? p[t] : v4f{0.f, 0.f, 0.f, 0.f};
                xv[4 * t + 0] = v[0]; xv[4 * t + 1] = v[1];
                xv[4 * t + 2] = v[2]; xv[4 * t + 3] = v[3];
            }
        } else {
#pragma unroll
            for (int s = 0; s < 16; ++s)
                xv[s] = (rowok && j0 + s < C) ? xr[j0 + s] : 0.f;
        }
        if (A_T) {
            if (VEC && full) {
                const v4f* p = reinterpret_cast<const v4f*>(ar + j0);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    v4f v = colok ? p[t] : v4f{0.f, 0.f, 0.f, 0.f};
                    av[4 * t + 0] = v[0]; av[4 * t + 1] = v[1];
                    av[4 * t + 2] = v[2]; av[4 * t + 3] = v[3];
                }
            } else {
#pragma unroll
                for (int s = 0; s < 16; ++s)
                    av[s] = (colok && j0 + s < C) ? ar[j0 + s] : 0.f;
            }
        } else {
#pragma unroll
            for (int s = 0; s < 16; ++s)
                av[s] = (colok && j0 + s < C) ? ar[(j0 + s) * lda] : 0.f;
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) acc = mfma32(xv[s], av[s], acc);
    }

#pragma unroll
    for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[r];
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * kWave; e += kThreads) {
        const int r = e / kWave, l = e % kWave;
        const float s = (red[0][r][l] + red[1][r][l]) + (red[2][r][l] + red[3][r][l]);
        const int col = l & 31;
        const int64_t row = row0 + acc_row(r, l);
        if (row < R) {
            if (DIRECT) {
                if (col < k) out[row * ldo + col] = s;
            } else {
                out[((int64_t)blockIdx.y * R + row) * 32 + col] = s;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Left sweep.  Workgroup = 128 columns of X; lane l loads the 4 consecutive
// columns 4 (l % 32) .. +3 of row i0 + (l / 32), and element t feeds the
// MFMA of accumulator tile t, whose M index (l % 32) stands for column
// col0 + 4 (l % 32) + t.  K runs over rows two at a time.  The 4 waves take
// interleaved 16-row blocks of the workgroup's row slice.
// ---------------------------------------------------------------------------
template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_sweep_left(
    int64_t R, int64_t C, const float* __restrict__ X, int64_t ldx, int k,
    const float* __restrict__ B, int64_t ldb, float* __restrict__ partial,
    int64_t blocks_per_split) {
    __shared__ float red[4][16][kWave];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int jl = lane & 31;
    const int kh = lane >> 5;
    const int64_t col0 = (int64_t)blockIdx.x * 128;
    const int64_t cb = col0 + 4 * jl;
    const int64_t nblocks = (R + 15) / 16;
    const int64_t b_begin = (int64_t)blockIdx.y * blocks_per_split;
    const int64_t b_end = min(nblocks, b_begin + blocks_per_split);
    const bool bcol = jl < k;
    const bool full4 = cb + 4 <= C;

    v16f acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;

    for (int64_t rb = b_begin + wave; rb < b_end; rb += 4) {
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int64_t i = rb * 16 + 2 * st + kh;
            const bool iok = i < R;
            const float* xr = X + (iok ? i : 0) * ldx;
            float x0, x1, x2, x3;
            if (VEC && full4) {
                v4f v = iok ? *reinterpret_cast<const v4f*>(xr + cb) : v4f{0.f, 0.f, 0.f, 0.f};
                x0 = v[0]; x1 = v[1]; x2 = v[2]; x3 = v[3];
            } else {
                x0 = (iok && cb + 0 < C) ? xr[cb + 0] : 0.f;
                x1 = (iok && cb + 1 < C) ? xr[cb + 1] : 0.f;
                x2 = (iok && cb + 2 < C) ? xr[cb + 2] : 0.f;
                x3 = (iok && cb + 3 < C) ? xr[cb + 3] : 0.f;
            }
            const float bv = (iok && bcol) ? B[i * ldb + jl] : 0.f;
            acc[0] = mfma32(x0, bv, acc[0]);
            acc[1] = mfma32(x1, bv, acc[1]);
            acc[2] = mfma32(x2, bv, acc[2]);
            acc[3] = mfma32(x3, bv, acc[3]);
        }
    }

    // Reduce the 4 waves, one accumulator tile at a time.
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[t][r];
        __syncthreads();
        for (int e = threadIdx.x; e < 16 * kWave; e += kThreads) {
            const int r = e / kWave, l = e % kWave;
            const float s = (red[0][r][l] + red[1][r][l]) + (red[2][r][l] + red[3][r][l]);
            const int c = l & 31;
            const int64_t col = col0 + 4 * acc_row(r, l) + t;
            if (col < C) partial[((int64_t)blockIdx.y * C + col) * 32 + c] = s;
        }
        __syncthreads();
    }
}

// out (rows x k) = sum over S slices of partial[s][rows][32]; optionally
// written transposed (k x rows).
__global__ __launch_bounds__(kThreads) void k_reduce_slices(
    int64_t rows, int k, int S, const float* __restrict__ partial, float* __restrict__ out,
    int64_t ldo, int trans) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= rows * 32) return;
    const int64_t r = e >> 5;
    const int c = (int)(e & 31);
    if (c >= k) return;
    float s = 0.f;
    for (int i = 0; i < S; ++i) s += partial[((int64_t)i * rows + r) * 32 + c];
    if (trans) out[(int64_t)c * ldo + r] = s;
    else out[r * ldo + c] = s;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Number of K slices: enough workgroups to cover every CU a few times, but
// at least 4 chunks (one per wave) per slice.
int64_t pick_splits(int64_t tiles, int64_t kunits, int num_cus) {
    const int64_t target = 4LL * num_cus;
    int64_t S = (target + tiles - 1) / tiles;
    const int64_t smax = kunits / 4 > 1 ? kunits / 4 : 1;
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    return S;
}

}  // namespace

size_t sweep_right_partial_floats(const Dev& d, int64_t R, int64_t C) {
    const int64_t tiles = (R + 31) / 32;
    const int64_t S = pick_splits(tiles, (C + 31) / 32, d.num_cus);
    return S > 1 ? (size_t)(S * R * 32) : 0;
}

hipError_t sweep_right(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx,
                       int k, const float* A, int64_t lda, bool a_trans, float* Y,
                       int64_t ldy, float* partial) {
    if (R <= 0 || k <= 0) return hipSuccess;
    const int64_t tiles = (R + 31) / 32;
    const int64_t nchunks = (C + 31) / 32;
    const int64_t S = pick_splits(tiles, nchunks, d.num_cus);
    const int64_t cps = (nchunks + S - 1) / S;
    const bool vec = (ldx % 4 == 0) && aligned16(X) &&
                     (!a_trans || ((lda % 4 == 0) && aligned16(A)));
    dim3 grid((unsigned)tiles, (unsigned)S);
    float* out = S > 1 ? partial : Y;
    const int64_t ldo = S > 1 ? 32 : ldy;
#define LAUNCH_R(AT, V, D) \
    hipLaunchKernelGGL((k_sweep_right<AT, V, D>), grid, dim3(kThreads), 0, d.stream, R, C, X, \
                       ldx, k, A, lda, out, ldo, cps)
    if (S > 1) {
        if (a_trans) { if (vec) LAUNCH_R(true, true, false); else LAUNCH_R(true, false, false); }
        else { if (vec) LAUNCH_R(false, true, false); else LAUNCH_R(false, false, false); }
    } else {
        if (a_trans) { if (vec) LAUNCH_R(true, true, true); else LAUNCH_R(true, false, true); }
        else { if (vec) LAUNCH_R(false, true, true); else LAUNCH_R(false, false, true); }
    }
#undef LAUNCH_R
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || S == 1) return e;
    const int64_t tot = R * 32;
    hipLaunchKernelGGL(k_reduce_slices, dim3((unsigned)((tot + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, d.stream, R, k, (int)S, partial, Y, ldy, 0);
    return hipGetLastError();
}

size_t sweep_left_partial_floats(const Dev& d, int64_t R, int64_t C) {
    const int64_t tiles = (C + 127) / 128;
    const int64_t S = pick_splits(tiles, (R + 15) / 16, d.num_cus);
    return (size_t)(S * C * 32);
}

hipError_t sweep_left(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx,
                      int k, const float* B, int64_t ldb, float* Z, int64_t ldz, bool z_trans,
                      float* partial) {
    if (C <= 0 || k <= 0) return hipSuccess;
    const int64_t tiles = (C + 127) / 128;
    const int64_t nblocks = (R + 15) / 16;
    const int64_t S = pick_splits(tiles, nblocks, d.num_cus);
    const int64_t bps = (nblocks + S - 1) / S;
    const bool vec = (ldx % 4 == 0) && aligned16(X);
    dim3 grid((unsigned)tiles, (unsigned)S);
    if (vec)
        hipLaunchKernelGGL(k_sweep_left<true>, grid, dim3(kThreads), 0, d.stream, R, C, X, ldx,
                           k, B, ldb, partial, bps);
    else
        hipLaunchKernelGGL(k_sweep_left<false>, grid, dim3(kThreads), 0, d.stream, R, C, X,
                           ldx, k, B, ldb, partial, bps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tot = C * 32;
    hipLaunchKernelGGL(k_reduce_slices, dim3((unsigned)((tot + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, d.stream, C, k, (int)S, partial, Z, ldz,
                       z_trans ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small utilities on X-sized or panel-sized data.
// ---------------------------------------------------------------------------
namespace {

__global__ __launch_bounds__(kThreads) void k_transpose(int64_t R, int64_t C,
                                                        const float* __restrict__ A, int64_t lda,
                                                        float* __restrict__ B, int64_t ldb) {
    __shared__ float tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int64_t r = r0 + j, c = c0 + tx;
        tile[j][tx] = (r < R && c < C) ? A[r * lda + c] : 0.f;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int64_t c = c0 + j, r = r0 + tx;
        if (c < C && r < R) B[c * ldb + r] = tile[tx][j];
    }
}

__global__ __launch_bounds__(kThreads) void k_check_input(int64_t R, int64_t C,
                                                          const float* __restrict__ X,
                                                          int64_t ldx, Control* ctl) {
    int bad = 0;
    const int64_t total = R * C;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t r = e / C, c = e - r * C;
        const float v = X[r * ldx + c];
        if (!isfinite(v)) bad |= CNMF_ST_NONFINITE;
        else if (v < 0.f) bad |= CNMF_ST_NEGATIVE;
    }
    if (__any(bad != 0)) {
        int w = bad;
        for (int off = 32; off >= 1; off >>= 1) w |= __shfl_xor(w, off, kWave);
        if ((threadIdx.x & 63) == 0) raise_status(ctl, w);
    }
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(kThreads) void k_to_bf16(int64_t R, int64_t C,
                                                      const float* __restrict__ X, int64_t ldx,
                                                      uint16_t* __restrict__ Xb, int64_t ldxb) {
    const int64_t total = R * C;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t r = e / C, c = e - r * C;
        Xb[r * ldxb + c] = f32_to_bf16_rne(X[r * ldx + c]);
    }
}

}  // namespace

hipError_t transpose(const Dev& d, int64_t R, int64_t C, const float* A, int64_t lda, float* B,
                     int64_t ldb) {
    if (R <= 0 || C <= 0) return hipSuccess;
    dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32));
    hipLaunchKernelGGL(k_transpose, grid, dim3(kThreads), 0, d.stream, R, C, A, lda, B, ldb);
    return hipGetLastError();
}

hipError_t check_input(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx,
                       Control* ctl) {
    if (R <= 0 || C <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_input, dim3((unsigned)(8 * d.num_cus)), dim3(kThreads), 0,
                       d.stream, R, C, X, ldx, ctl);
    return hipGetLastError();
}

hipError_t to_bf16(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx,
                   uint16_t* Xb, int64_t ldxb) {
    if (R <= 0 || C <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)(8 * d.num_cus)), dim3(kThreads), 0, d.stream,
                       R, C, X, ldx, Xb, ldxb);
    return hipGetLastError();
}

}  // namespace cnmf
