// BF16 form of the X-sized sweeps: X stored as bfloat16, the skinny operand
// rounded to bfloat16 (round to nearest even), products on the matrix cores
// (v_mfma_f32_32x32x8_bf16, FP32 accumulation).  Same products as the FP32
// sweeps (Algorithm 2's X Omega, X^T Q, Q^T X, X Q), half the HBM bytes.
//
// v_mfma_f32_32x32x8_bf16 operand layout: lane l holds four bf16 values,
// A[m = l % 32][k = 4 (l / 32) + i] and B[k = 4 (l / 32) + i][n = l % 32],
// i = 0..3; the accumulator layout is that of the FP32 32x32 instruction.
// Only the pairing of A and B elements on the same (lane, i) matters for
// the sum, so each kernel assigns its own reduction index to (l / 32, i).
#include "internal.hpp"

namespace cnmf {

namespace {

constexpr int kThreads = 256;
typedef short v4s __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v16f mfma_bf16(v4s a, v4s b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int acc_row(int r, int lane) {
    return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

__device__ __forceinline__ v4s as_v4s(unsigned lo, unsigned hi) {
    v4s v;
    v[0] = (short)(lo & 0xffffu);
    v[1] = (short)(lo >> 16);
    v[2] = (short)(hi & 0xffffu);
    v[3] = (short)(hi >> 16);
    return v;
}

constexpr int kSW = 256;            // bf16 columns per right-sweep stage
constexpr int kPB = kSW + 8;        // LDS row pitch (bf16): rows 4 banks apart

// ---------------------------------------------------------------------------
// Panel: PT[n][c] = bf16(A[c][n]) (or bf16(AT[n][c])) for n < k, c < C, zero
// elsewhere up to 32 x ldp; ldp is C rounded up to a stage, so full-stage
// loads of the panel never leave it and padding contributes zero.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_pack_panel(int64_t C, int k, const float* __restrict__ A,
                                                         int64_t lda, int a_trans,
                                                         uint16_t* __restrict__ PT, int64_t ldp) {
    const int64_t total = 32 * ldp;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const int n = (int)(e / ldp);
        const int64_t c = e - (int64_t)n * ldp;
        float v = 0.f;
        if (n < k && c < C) v = a_trans ? A[(int64_t)n * lda + c] : A[c * lda + n];
        PT[e] = f32_to_bf16_rne(v);
    }
}

// ---------------------------------------------------------------------------
// Right sweep, Y = X A.  Workgroup = 32 rows times one column slice.  Stages
// of 32 rows x 256 bf16 columns go through LDS; each wave loads 8 rows with
// four 1 KB instructions (two 512-byte row pieces each) and prefetches the
// next stage while the current one is multiplied.  Wave w multiplies stage
// columns 64 w .. 64 w + 63: lane half g = l / 32 takes 32 of them, and MFMA s
// takes columns 4 s .. 4 s + 3 of that range (A from the LDS row l % 32, B
// from the packed panel row l % 32).  The four waves' sums meet in LDS.
// ---------------------------------------------------------------------------
template <bool DIRECT, bool VEC>
__global__ __launch_bounds__(kThreads) void k_sweep_right_bf16(
    int64_t R, int64_t C, const uint16_t* __restrict__ X, int64_t ldx, int k,
    const uint16_t* __restrict__ PT, int64_t ldp, float* __restrict__ out, int64_t ldo,
    int64_t span) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[32 * kPB];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 5;
    const int64_t row0 = (int64_t)blockIdx.x * 32;
    const int64_t c_lo = (int64_t)blockIdx.y * span;
    const int64_t c_hi = min(C, c_lo + span);
    const int64_t nst = (c_hi - c_lo + kSW - 1) / kSW;
    const int64_t nfull = VEC ? (c_hi - c_lo) / kSW : 0;
    const int koff = 64 * wave + 32 * g;           // this lane's 32 stage columns
    const int xcol = 8 * (lane & 31);               // this lane's 8 load columns
    const uint16_t* prow = PT + (int64_t)(lane & 31) * ldp;

    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    v4u xn[4], bn[4], bc[4];

    auto load_b = [&](int64_t cb) {
        const v4u* p = reinterpret_cast<const v4u*>(prow + cb + koff);
#pragma unroll
        for (int t = 0; t < 4; ++t) bn[t] = p[t];
    };
    auto load_fast = [&](int64_t st) {
        st = st < nfull ? st : nfull - 1;
        const int64_t cb = c_lo + kSW * st;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int64_t row = row0 + 8 * wave + 2 * rr + g;
            const uint16_t* xr = X + (row < R ? row : R - 1) * ldx;
            xn[rr] = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(xr + cb + xcol));
        }
        load_b(cb);
    };
    auto load_slow = [&](int64_t st) {
        const int64_t cb = c_lo + kSW * st;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int64_t row = row0 + 8 * wave + 2 * rr + g;
            const uint16_t* xr = X + (row < R ? row : R - 1) * ldx;
            unsigned w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t c0 = cb + xcol + 2 * u, c1 = c0 + 1;
                const unsigned lo = c0 < c_hi ? xr[c0] : 0u;
                const unsigned hi = c1 < c_hi ? xr[c1 < c_hi ? c1 : c0] : 0u;
                w[u] = lo | (hi << 16);
            }
            xn[rr] = v4u{w[0], w[1], w[2], w[3]};
        }
        load_b(cb);
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
            *reinterpret_cast<v4u*>(&xs[(8 * wave + 2 * rr + g) * kPB + xcol]) = xn[rr];
#pragma unroll
        for (int t = 0; t < 4; ++t) bc[t] = bn[t];
    };
    auto compute = [&]() {
        const v4u* xr = reinterpret_cast<const v4u*>(&xs[(lane & 31) * kPB + koff]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const v4u a = xr[t];
            acc = mfma_bf16(as_v4s(a[0], a[1]), as_v4s(bc[t][0], bc[t][1]), acc);
            acc = mfma_bf16(as_v4s(a[2], a[3]), as_v4s(bc[t][2], bc[t][3]), acc);
        }
    };

    if (nfull > 0) {
        load_fast(0);
        store_stage();
        __syncthreads();
        for (int64_t st = 0; st < nfull; ++st) {
            load_fast(st + 1);
            __builtin_amdgcn_sched_barrier(0);
            compute();
            __builtin_amdgcn_sched_barrier(0);
            __syncthreads();
            store_stage();
            __syncthreads();
        }
    }
    for (int64_t st = nfull; st < nst; ++st) {
        __syncthreads();
        load_slow(st);
        store_stage();
        __syncthreads();
        compute();
    }
    __syncthreads();

    float* red = reinterpret_cast<float*>(xs);     // 4 waves x 16 x 64 floats = 16 KB
#pragma unroll
    for (int r = 0; r < 16; ++r) red[(wave * 16 + r) * 64 + lane] = acc[r];
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * 64; e += kThreads) {
        const int r = e / 64, l = e % 64;
        const float s = (red[r * 64 + l] + red[(16 + r) * 64 + l]) +
                        (red[(32 + r) * 64 + l] + red[(48 + r) * 64 + l]);
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
// Left sweep, Z = X^T B, without LDS staging, on v_mfma_f32_32x32x16_bf16
// (lane l holds eight bf16 values: A[m = l % 32][k = 8 (l / 32) + i],
// B[k = 8 (l / 32) + i][n = l % 32]).  A wave owns 256 columns of X.  Load
// instruction i covers two rows (lanes 0-31 the first, lanes 32-63 the
// second) x 256 columns, 16 bytes per lane, so lanes l and l + 32 hold the
// same 8 columns of different rows.  After eight instructions (rows
// r0 + g + 2 i, g = l / 32, i = 0..7) lane l has, for each of its columns,
// the eight values that reduction slots (g, i) need: MFMA j (j = 0..7) takes
// column 8 (l % 32) + j as its M index l % 32, so one group of sixteen rows
// feeds eight MFMAs with no data exchange.  The B operand is
// bf16(B[r0 + g + 2 i][n = l % 32]).  The four waves of a workgroup take
// interleaved row groups of the slice and are summed through LDS in wave
// order.
// ---------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v16f mfma_bf16_x16(v4u_t a, v4u_t b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

constexpr int kLG = 16;     // rows per group (two per load instruction)

template <bool VEC>
__global__ __launch_bounds__(kThreads, 2) void k_sweep_left_bf16(
    int64_t R, int64_t C, const uint16_t* __restrict__ X, int64_t ldx, int k,
    const float* __restrict__ B, int64_t ldb, float* __restrict__ partial, int64_t rspan) {
    __shared__ float red[8 * 16 * 64];        // 32 KB: one wave's accumulators
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 5;
    const int n = lane & 31;
    const int nc = n < k ? n : 0;
    const int64_t col0 = (int64_t)blockIdx.x * 256;
    const int64_t r_lo = (int64_t)blockIdx.y * rspan;
    const int64_t r_hi = min(R, r_lo + rspan);
    const int64_t ngr = (r_hi - r_lo + kLG - 1) / kLG;   // row groups in the slice
    const int64_t col = col0 + 8 * n;
    const bool full = VEC && col0 + 256 <= C;            // uniform across the workgroup

    v16f acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;

    v4u xn[8], xc[8];
    float bn[8], bc[8];          // raw B values; rounded and masked at use
    int64_t bn_row0 = 0, bc_row0 = 0;
    auto load_b = [&](int64_t rb) {
        bn_row0 = rb;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t row = rb + g + 2 * i;
            bn[i] = B[(row < R ? row : R - 1) * ldb + nc];
        }
    };
    auto load_fast = [&](int64_t gi) {
        gi = gi < ngr ? gi : ngr - 1;
        const int64_t rb = r_lo + kLG * gi;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t row = rb + g + 2 * i;
            const uint16_t* xr = X + (row < R ? row : R - 1) * ldx;
            xn[i] = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(xr + col));
        }
        load_b(rb);
    };
    auto load_slow = [&](int64_t gi) {
        const int64_t rb = r_lo + kLG * gi;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t row = rb + g + 2 * i;
            const uint16_t* xr = X + (row < R ? row : R - 1) * ldx;
            unsigned w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t c0 = col + 2 * u, c1 = c0 + 1;
                const unsigned lo = c0 < C ? xr[c0] : 0u;
                const unsigned hi = c1 < C ? xr[c1] : 0u;
                w[u] = lo | (hi << 16);
            }
            xn[i] = v4u{w[0], w[1], w[2], w[3]};
        }
        load_b(rb);
    };
    auto take = [&]() {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            xc[i] = xn[i];
            bc[i] = bn[i];
        }
        bc_row0 = bn_row0;
    };
    auto compute = [&]() {
        unsigned h[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const bool live = bc_row0 + g + 2 * i < r_hi && n < k;
            h[i] = live ? f32_to_bf16_rne(bc[i]) : 0u;
        }
        const v4u_t b = v4u_t{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                              h[6] | (h[7] << 16)};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int d = j >> 1;
            v4u_t a;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const unsigned x0 = xc[2 * p][d], x1 = xc[2 * p + 1][d];
                a[p] = (j & 1) ? ((x0 >> 16) | (x1 & 0xffff0000u)) : ((x0 & 0xffffu) | (x1 << 16));
            }
            acc[j] = mfma_bf16_x16(a, b, acc[j]);
        }
    };

    // wave w takes groups w, w + 4, ...
    const int64_t mine = ngr > wave ? (ngr - wave + 3) / 4 : 0;
    if (full) {
        if (mine > 0) {
            load_fast(wave);
            for (int64_t t = 0; t < mine; ++t) {
                take();
                load_fast(wave + 4 * (t + 1));
                __builtin_amdgcn_sched_barrier(0);
                compute();
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        for (int64_t t = 0; t < mine; ++t) {
            load_slow(wave + 4 * t);
            take();
            compute();
        }
    }

    // ((w0 + w1) + w2) + w3 through LDS, then the last wave writes the slice
    for (int w2 = 0; w2 < 4; ++w2) {
        if (wave == w2) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    float v = acc[j][r];
                    float* slot = &red[(j * 16 + r) * 64 + lane];
                    if (w2 > 0) v = *slot + v;
                    if (w2 < 3) {
                        *slot = v;
                    } else if (n < k) {
                        const int64_t c = col0 + 8 * acc_row(r, lane) + j;
                        if (c < C) partial[((int64_t)blockIdx.y * C + c) * 32 + n] = v;
                    }
                }
        }
        __syncthreads();
    }
}

template <class K>
int occupancy(K kernel) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(kernel),
                                                     kThreads, 0) != hipSuccess || blocks < 1)
        blocks = 1;
    return blocks;
}

struct Plan { int64_t tiles, S, span; };

Plan right_plan(const Dev& d, int64_t R, int64_t C) {
    static const int occ = occupancy(k_sweep_right_bf16<false, true>);
    Plan p;
    p.tiles = (R + 31) / 32;
    const int64_t stages = (C + kSW - 1) / kSW;
    p.S = pick_splits(p.tiles, stages, d.num_cus, occ);
    p.span = kSW * ((stages + p.S - 1) / p.S);
    p.S = (C + p.span - 1) / p.span;
    return p;
}

Plan left_plan(const Dev& d, int64_t R, int64_t C) {
    static const int occ = occupancy(k_sweep_left_bf16<true>);
    Plan p;
    p.tiles = (C + 255) / 256;
    const int64_t groups = (R + 4 * kLG - 1) / (4 * kLG);   // 4 waves x 16 rows per round
    p.S = pick_splits(p.tiles, groups, d.num_cus, occ);
    p.span = 4 * kLG * ((groups + p.S - 1) / p.S);
    p.S = (R + p.span - 1) / p.span;
    return p;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

size_t bf16_pack_elems(int64_t C) { return (size_t)32 * (size_t)((C + kSW - 1) / kSW * kSW); }

size_t sweep_right_bf16_partial_floats(const Dev& d, int64_t R, int64_t C) {
    const Plan p = right_plan(d, R, C);
    return p.S > 1 ? (size_t)(p.S * R * 32) : 0;
}

size_t sweep_left_bf16_partial_floats(const Dev& d, int64_t R, int64_t C) {
    const Plan p = left_plan(d, R, C);
    return (size_t)(p.S * C * 32);
}

hipError_t sweep_right_bf16(const Dev& d, int64_t R, int64_t C, const uint16_t* Xb, int64_t ldx,
                            int k, const float* A, int64_t lda, bool a_trans, float* Y,
                            int64_t ldy, float* partial, uint16_t* pack) {
    if (R <= 0 || C <= 0 || k <= 0) return hipSuccess;
    const int64_t ldp = (C + kSW - 1) / kSW * kSW;
    hipLaunchKernelGGL(k_pack_panel, dim3((unsigned)std::min<int64_t>(4 * d.num_cus, (32 * ldp + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, d.stream, C, k, A, lda, a_trans ? 1 : 0, pack, ldp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool vec = ldx % 8 == 0 && aligned16(Xb);
    const Plan p = right_plan(d, R, C);
    const bool direct = p.S == 1;
    float* out = direct ? Y : partial;
    const int64_t ldo = direct ? ldy : 32;
    dim3 grid((unsigned)p.tiles, (unsigned)p.S);
#define LAUNCH_RB(D, V)                                                                        \
    hipLaunchKernelGGL((k_sweep_right_bf16<D, V>), grid, dim3(kThreads), 0, d.stream, R, C, Xb, \
                       ldx, k, pack, ldp, out, ldo, p.span)
    if (direct) { if (vec) LAUNCH_RB(true, true); else LAUNCH_RB(true, false); }
    else { if (vec) LAUNCH_RB(false, true); else LAUNCH_RB(false, false); }
#undef LAUNCH_RB
    e = hipGetLastError();
    if (e != hipSuccess || direct) return e;
    return reduce_slices(d, R, k, p.S, 32, partial, Y, ldy, false);
}

hipError_t sweep_left_bf16(const Dev& d, int64_t R, int64_t C, const uint16_t* Xb, int64_t ldx,
                           int k, const float* B, int64_t ldb, float* Z, int64_t ldz,
                           bool z_trans, float* partial) {
    if (R <= 0 || C <= 0 || k <= 0) return hipSuccess;
    const bool vec = ldx % 8 == 0 && aligned16(Xb);
    const Plan p = left_plan(d, R, C);
    dim3 grid((unsigned)p.tiles, (unsigned)p.S);
    if (vec)
        hipLaunchKernelGGL((k_sweep_left_bf16<true>), grid, dim3(kThreads), 0, d.stream, R, C, Xb,
                           ldx, k, B, ldb, partial, p.span);
    else
        hipLaunchKernelGGL((k_sweep_left_bf16<false>), grid, dim3(kThreads), 0, d.stream, R, C,
                           Xb, ldx, k, B, ldb, partial, p.span);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_slices(d, C, k, p.S, 32, partial, Z, ldz, z_trans);
}

}  // namespace cnmf
