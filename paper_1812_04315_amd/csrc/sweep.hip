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
#include <cstdlib>

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

__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Right sweep, Y = X A.  Workgroup = 32 rows of X times one K slice.
// X is streamed in stages of 32 rows x SW columns: each wave reads 8 rows
// of it, a contiguous kilobyte per instruction (one row when SW = 256, two
// half rows when SW = 128), into LDS; the next stage is loaded into
// registers while the current one is multiplied.  Wave w multiplies the
// quarter KW = SW / 4 columns starting at KW w.
//   NT = 32 (k > 16): v_mfma_f32_32x32x2f32.  Lane l reads row l % 32 and NA
//     consecutive columns starting at KW w + NA (l / 32); MFMA s uses element
//     s, so its K index (l / 32) stands for that start + s, and its B operand
//     is A at that column and output column l % 32.
//   NT = 16 (k <= 16): v_mfma_f32_16x16x4f32 on two 16-row tiles, lane l at
//     rows l % 16 and 16 + l % 16, columns KW w + NA (l / 16) + s.
// The four waves' partial sums are added through LDS at the end.
// ---------------------------------------------------------------------------
template <int NT, int SW>
struct RightShape {
    static constexpr int KW = SW / 4;                 // K columns per wave per stage
    static constexpr int KL = NT == 32 ? 2 : 4;       // K lane groups of the MFMA
    static constexpr int NA = KW / KL;                // A values per lane per stage
    static constexpr int PITCH = SW + 4;              // LDS row pitch (bank spread)
    static constexpr int XV = SW / 32;                // float4 X loads per lane per stage
};

template <int NT, int SW, bool A_T, bool VEC>
__device__ __forceinline__ void right_load_a(const float* __restrict__ A, int64_t lda, int k,
                                             int64_t K0, int lane, float (&a)[RightShape<NT, SW>::NA]) {
    constexpr int NA = RightShape<NT, SW>::NA;
    const int n = NT == 32 ? (lane & 31) : (lane & 15);
    const int nc = n < k ? n : 0;
    if (A_T && VEC) {
        const v4f* p = reinterpret_cast<const v4f*>(A + nc * lda + K0);
#pragma unroll
        for (int t = 0; t < NA / 4; ++t) {
            const v4f v = p[t];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[4 * t + u] = v[u];
        }
    } else if (A_T) {
#pragma unroll
        for (int s = 0; s < NA; ++s) a[s] = A[nc * lda + K0 + s];
    } else {
#pragma unroll
        for (int s = 0; s < NA; ++s) a[s] = A[(K0 + s) * lda + nc];
    }
}

template <int NT, int SW, bool A_T, bool DIRECT, bool VEC>
__device__ __forceinline__ void right_body(
    int64_t R, int64_t C, const float* __restrict__ X, int64_t ldx, int k,
    const float* __restrict__ A, int64_t lda, float* __restrict__ out, int64_t ldo,
    int64_t span, const int64_t tile, const int64_t slice) {
    using Sh = RightShape<NT, SW>;
    constexpr int KW = Sh::KW, NA = Sh::NA, PITCH = Sh::PITCH, XV = Sh::XV;
    __shared__ __attribute__((aligned(16))) float xs[32 * PITCH > 4096 ? 32 * PITCH : 4096];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t row0 = tile * 32;
    const int64_t c_lo = slice * span;
    const int64_t c_hi = min(C, c_lo + span);
    const int64_t nst = (c_hi - c_lo + SW - 1) / SW;
    const int koff = KW * wave + NA * (NT == 32 ? (lane >> 5) : (lane >> 4));
    // X loads: instruction rr covers row 8 w + rr (SW = 256) or rows
    // 8 w + 2 rr + l / 32 (SW = 128); lane column offset within the stage:
    const int xrow_l = SW == 256 ? 0 : (lane >> 5);
    const int xcol_l = SW == 256 ? 4 * lane : 4 * (lane & 31);
    const int xrow_step = SW == 256 ? 1 : 2;

    v16f acc32;
    v4f acc16[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc32[r] = 0.f;
    acc16[0] = acc16[1] = v4f{0.f, 0.f, 0.f, 0.f};

    v4f xn[XV];
    float an[NA], ac[NA];
    // Full stages (inside the slice, aligned rows) use plain vector loads;
    // a ragged last stage, or unaligned rows, use clamped scalar loads that
    // zero what lies past the slice.  The two never share a loop, so the
    // pipelined loop has a single load path and nothing waits early.
    const int64_t nfull = VEC ? (c_hi - c_lo) / SW : 0;
    auto load_fast = [&](int64_t st) {
        st = st < nfull ? st : nfull - 1;
        const int64_t cb = c_lo + SW * st;
#pragma unroll
        for (int rr = 0; rr < XV; ++rr) {
            const int64_t row = row0 + 8 * wave + xrow_step * rr + xrow_l;
            const float* xr = X + (row < R ? row : R - 1) * ldx;
            xn[rr] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(xr + cb + xcol_l));
        }
        right_load_a<NT, SW, A_T, VEC>(A, lda, k, cb + koff, lane, an);
    };
    auto load_slow = [&](int64_t st) {
        const int64_t cb = c_lo + SW * st;
        const int64_t K0 = cb + koff;
#pragma unroll
        for (int rr = 0; rr < XV; ++rr) {
            const int64_t row = row0 + 8 * wave + xrow_step * rr + xrow_l;
            const float* xr = X + (row < R ? row : R - 1) * ldx;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t c = cb + xcol_l + u;
                const float v = xr[c < c_hi ? c : c_hi - 1];
                xn[rr][u] = c < c_hi ? v : 0.f;
            }
        }
        const int n = NT == 32 ? (lane & 31) : (lane & 15);
        const int nc = n < k ? n : 0;
#pragma unroll
        for (int s = 0; s < NA; ++s) {
            const int64_t kk = K0 + s;
            const int64_t kc = kk < c_hi ? kk : c_hi - 1;
            const float v = A_T ? A[nc * lda + kc] : A[kc * lda + nc];
            an[s] = kk < c_hi ? v : 0.f;
        }
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int rr = 0; rr < XV; ++rr)
            *reinterpret_cast<v4f*>(&xs[(8 * wave + xrow_step * rr + xrow_l) * PITCH + xcol_l]) = xn[rr];
#pragma unroll
        for (int s = 0; s < NA; ++s) ac[s] = an[s];
    };
    auto compute = [&]() {
        if (NT == 32) {
            const float* xr = &xs[(lane & 31) * PITCH + koff];
#pragma unroll
            for (int t = 0; t < NA / 4; ++t) {
                const v4f v = *reinterpret_cast<const v4f*>(xr + 4 * t);
#pragma unroll
                for (int u = 0; u < 4; ++u) acc32 = mfma32(v[u], ac[4 * t + u], acc32);
            }
        } else {
#pragma unroll
            for (int t = 0; t < NA / 4; ++t) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    const v4f v = *reinterpret_cast<const v4f*>(
                        &xs[(16 * mt + (lane & 15)) * PITCH + koff + 4 * t]);
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc16[mt] = mfma16(v[u], ac[4 * t + u], acc16[mt]);
                }
            }
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

    // Sum the four waves through LDS (reusing the stage buffer).
    float* red = xs;
    if (NT == 32) {
#pragma unroll
        for (int r = 0; r < 16; ++r) red[(wave * 16 + r) * 64 + lane] = acc32[r];
    } else {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[(wave * 16 + mt * 4 + i) * 64 + lane] = acc16[mt][i];
    }
    __syncthreads();
    // NT = 32: 16 accumulator registers per lane; NT = 16: 2 tiles x 4.
    constexpr int NREG = NT == 32 ? 16 : 8;
    for (int e = threadIdx.x; e < NREG * 64; e += kThreads) {
        const int r = e / 64, l = e % 64;
        const float s = (red[r * 64 + l] + red[(16 + r) * 64 + l]) +
                        (red[(32 + r) * 64 + l] + red[(48 + r) * 64 + l]);
        int col, rloc;
        if (NT == 32) {
            col = l & 31;
            rloc = acc_row(r, l);
        } else {
            col = l & 15;
            rloc = 16 * (r >> 2) + 4 * (l >> 4) + (r & 3);
        }
        const int64_t row = row0 + rloc;
        if (row < R) {
            if (DIRECT) {
                if (col < k) out[row * ldo + col] = s;
            } else {
                out[(slice * R + row) * NT + col] = s;
            }
        }
    }
}

template <int NT, int SW, bool A_T, bool DIRECT, bool VEC>
__global__ __launch_bounds__(kThreads) void k_sweep_right(
    int64_t R, int64_t C, const float* __restrict__ X, int64_t ldx, int k,
    const float* __restrict__ A, int64_t lda, float* __restrict__ out, int64_t ldo,
    int64_t span) {
    right_body<NT, SW, A_T, DIRECT, VEC>(R, C, X, ldx, k, A, lda, out, ldo, span, blockIdx.x,
                                         blockIdx.y);
}

// ---------------------------------------------------------------------------
// Left sweep, Z = X^T B.  Workgroup = 256 columns of X times one row slice.
// X is streamed in stages of 16 rows x 256 columns (each wave reads 4 rows,
// one contiguous kilobyte per row and instruction) through LDS; the next
// stage is in registers while the current one is multiplied.  Wave w owns
// columns 64 w .. 64 w + 63 of the block, so no reduction across waves is
// needed.  The M index of the MFMA is the column of X, K the row, N the
// column of B.
//   NT = 32: v_mfma_f32_32x32x2f32, two 32-column tiles per wave, K = 2 rows.
//   NT = 16: v_mfma_f32_16x16x4f32, four 16-column tiles per wave, K = 4 rows.
// ---------------------------------------------------------------------------
constexpr int kLPad = 272;   // row pitch: 4-row groups of 16 floats hit distinct banks

template <int NT, bool VEC>
__device__ __forceinline__ void left_body(
    int64_t R, int64_t C, const float* __restrict__ X, int64_t ldx, int k,
    const float* __restrict__ B, int64_t ldb, float* __restrict__ partial, int64_t rspan,
    const int64_t tile, const int64_t slice) {
    __shared__ __attribute__((aligned(16))) float xs[16 * kLPad];
    constexpr int KS = NT == 32 ? 8 : 4;        // K steps per stage
    constexpr int MT = NT == 32 ? 2 : 4;        // M tiles per wave
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t col0 = tile * 256;
    const int64_t r_lo = slice * rspan;
    const int64_t r_hi = min(R, r_lo + rspan);
    const int64_t nst = (r_hi - r_lo + 15) / 16;
    const int n = NT == 32 ? (lane & 31) : (lane & 15);
    const int nc = n < k ? n : 0;
    const int kl = NT == 32 ? (lane >> 5) : (lane >> 4);   // K index within an MFMA

    v16f acc32[MT];
    v4f acc16[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc32[t][r] = 0.f;
        acc16[t] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    v4f xn[4];
    float bn[KS], bc[KS];
    int64_t bn_row0 = 0, bc_row0 = 0;
    const int64_t col = col0 + 4 * lane;
    const bool full = VEC && col0 + 256 <= C;   // uniform across the workgroup
    auto load_b = [&](int64_t rb) {
        bn_row0 = rb;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int64_t row = rb + (NT == 32 ? 2 : 4) * s + kl;
            bn[s] = B[(row < R ? row : R - 1) * ldb + nc];
        }
    };
    auto load_fast = [&](int64_t st) {
        st = st < nst ? st : nst - 1;
        const int64_t rb = r_lo + 16 * st;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int64_t row = rb + 4 * wave + rr;
            const float* xr = X + (row < R ? row : R - 1) * ldx;
            xn[rr] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(xr + col));
        }
        load_b(rb);
    };
    auto load_slow = [&](int64_t st) {
        const int64_t rb = r_lo + 16 * st;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int64_t row = rb + 4 * wave + rr;
            const float* xr = X + (row < R ? row : R - 1) * ldx;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t c = col + u;
                const float v = xr[c < C ? c : C - 1];
                xn[rr][u] = c < C ? v : 0.f;
            }
        }
        load_b(rb);
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
            *reinterpret_cast<v4f*>(&xs[(4 * wave + rr) * kLPad + 4 * lane]) = xn[rr];
#pragma unroll
        for (int s = 0; s < KS; ++s) bc[s] = bn[s];
        bc_row0 = bn_row0;
    };
    auto compute = [&]() {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int rr = (NT == 32 ? 2 : 4) * s + kl;
            const float bv = (bc_row0 + rr < r_hi) ? bc[s] : 0.f;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const float av = xs[rr * kLPad + 64 * wave + NT * t + n];
                if (NT == 32) acc32[t] = mfma32(av, bv, acc32[t]);
                else acc16[t] = mfma16(av, bv, acc16[t]);
            }
        }
    };

    if (nst > 0 && full) {
        load_fast(0);
        store_stage();
        __syncthreads();
        for (int64_t st = 0; st < nst; ++st) {
            load_fast(st + 1);
            __builtin_amdgcn_sched_barrier(0);
            compute();
            __builtin_amdgcn_sched_barrier(0);
            __syncthreads();
            store_stage();
            __syncthreads();
        }
    } else {
        for (int64_t st = 0; st < nst; ++st) {
            __syncthreads();
            load_slow(st);
            store_stage();
            __syncthreads();
            compute();
        }
    }

#pragma unroll
    for (int t = 0; t < MT; ++t) {
        if (NT == 32) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t c = col0 + 64 * wave + 32 * t + acc_row(r, lane);
                if (c < C) partial[(slice * C + c) * NT + (lane & 31)] = acc32[t][r];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t c = col0 + 64 * wave + 16 * t + 4 * (lane >> 4) + i;
                if (c < C) partial[(slice * C + c) * NT + (lane & 15)] = acc16[t][i];
            }
        }
    }
}

template <int NT, bool VEC>
__global__ __launch_bounds__(kThreads) void k_sweep_left(
    int64_t R, int64_t C, const float* __restrict__ X, int64_t ldx, int k,
    const float* __restrict__ B, int64_t ldb, float* __restrict__ partial, int64_t rspan) {
    left_body<NT, VEC>(R, C, X, ldx, k, B, ldb, partial, rspan, blockIdx.x, blockIdx.y);
}

// out (rows x k) = sum over S slices of partial[s][rows][nt]; optionally
// written transposed (k x rows).
__global__ __launch_bounds__(kThreads) void k_reduce_slices(
    int64_t rows, int k, int S, int nt, const float* __restrict__ partial, float* __restrict__ out,
    int64_t ldo, int trans) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= rows * nt) return;
    const int64_t r = e / nt;
    const int c = (int)(e % nt);
    if (c >= k) return;
    float s = 0.f;
    for (int i = 0; i < S; ++i) s += partial[((int64_t)i * rows + r) * nt + c];
    if (trans) out[(int64_t)c * ldo + r] = s;
    else out[r * ldo + c] = s;
}

template <class K>
int occupancy(K kernel) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(kernel),
                                                     kThreads, 0) != hipSuccess || blocks < 1)
        blocks = 1;
    return blocks;
}

int right_sw() {
    static const int v = [] {
        const char* e = std::getenv("CNMF_RSW");
        return (e && std::atoi(e) == 256) ? 256 : 128;
    }();
    return v;
}

int occ_right(int nt) {
    static const int v16_128 = occupancy(k_sweep_right<16, 128, true, false, true>);
    static const int v32_128 = occupancy(k_sweep_right<32, 128, true, false, true>);
    static const int v16_256 = occupancy(k_sweep_right<16, 256, true, false, true>);
    static const int v32_256 = occupancy(k_sweep_right<32, 256, true, false, true>);
    if (right_sw() == 128) return nt == 16 ? v16_128 : v32_128;
    return nt == 16 ? v16_256 : v32_256;
}

int occ_left() {
    static const int v = occupancy(k_sweep_left<32, true>);
    return v;
}

struct RightPlan { int64_t tiles, S, span; int nt, sw; };
RightPlan right_plan(const Dev& d, int64_t R, int64_t C, int k) {
    RightPlan p;
    p.nt = k <= 16 ? 16 : 32;
    p.sw = right_sw();
    p.tiles = (R + 31) / 32;
    const int64_t stages = (C + p.sw - 1) / p.sw;
    p.S = pick_splits(p.tiles, stages, d.num_cus, occ_right(p.nt));
    p.span = p.sw * ((stages + p.S - 1) / p.S);
    p.S = (C + p.span - 1) / p.span;
    return p;
}

struct LeftPlan { int64_t tiles, S, rspan; int nt; };
LeftPlan left_plan(const Dev& d, int64_t R, int64_t C, int k) {
    LeftPlan p;
    p.nt = k <= 16 ? 16 : 32;
    p.tiles = (C + 255) / 256;
    const int64_t stages = (R + 15) / 16;
    p.S = pick_splits(p.tiles, stages, d.num_cus, occ_left());
    p.rspan = 16 * ((stages + p.S - 1) / p.S);
    p.S = (R + p.rspan - 1) / p.rspan;
    return p;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// ---------------------------------------------------------------------------
// Batched launches: one workgroup per work item, any mix of instances.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_sweep_right_batched(const SweepDesc* __restrict__ desc,
                                                                 const WorkItem* __restrict__ work) {
    const WorkItem w = work[blockIdx.x];
    const SweepDesc& s = desc[w.inst];
    const int64_t tile = w.item % s.tiles, slice = w.item / s.tiles;
    if (s.nt == 16)
        right_body<16, 128, true, false, true>(s.R, s.C, s.X, s.ldx, s.k, s.A, s.lda, s.partial,
                                               16, s.span, tile, slice);
    else
        right_body<32, 128, true, false, true>(s.R, s.C, s.X, s.ldx, s.k, s.A, s.lda, s.partial,
                                               32, s.span, tile, slice);
}

__global__ __launch_bounds__(kThreads) void k_sweep_left_batched(const SweepDesc* __restrict__ desc,
                                                                const WorkItem* __restrict__ work) {
    const WorkItem w = work[blockIdx.x];
    const SweepDesc& s = desc[w.inst];
    const int64_t tile = w.item % s.tiles, slice = w.item / s.tiles;
    if (s.nt == 16)
        left_body<16, true>(s.R, s.C, s.X, s.ldx, s.k, s.A, s.lda, s.partial, s.span, tile, slice);
    else
        left_body<32, true>(s.R, s.C, s.X, s.ldx, s.k, s.A, s.lda, s.partial, s.span, tile, slice);
}

// Slice sums of one 256-element chunk of an instance's partial output.
__global__ __launch_bounds__(kThreads) void k_reduce_batched(const SweepDesc* __restrict__ desc,
                                                            const WorkItem* __restrict__ work,
                                                            int left) {
    const WorkItem w = work[blockIdx.x];
    const SweepDesc& s = desc[w.inst];
    const int64_t rows = left ? s.C : s.R;
    const int64_t e = (int64_t)w.item * kThreads + threadIdx.x;
    if (e >= rows * s.nt) return;
    const int64_t r = e / s.nt;
    const int c = (int)(e % s.nt);
    if (c >= s.k) return;
    float v = 0.f;
    for (int i = 0; i < s.S; ++i) v += s.partial[((int64_t)i * rows + r) * s.nt + c];
    if (s.trans) s.Y[(int64_t)c * s.ldy + r] = v;
    else s.Y[r * s.ldy + c] = v;
}

__global__ __launch_bounds__(kThreads) void k_transpose_batched(const TransDesc* __restrict__ desc,
                                                               const WorkItem* __restrict__ work) {
    __shared__ float tile[32][33];
    const WorkItem w = work[blockIdx.x];
    const TransDesc& t = desc[w.inst];
    const int64_t tc = (t.C + 31) / 32;
    const int64_t r0 = (w.item / tc) * 32, c0 = (w.item % tc) * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int j = ty; j < 32; j += 8) {
        const int64_t r = r0 + j, c = c0 + tx;
        tile[j][tx] = (r < t.R && c < t.C) ? t.A[r * t.lda + c] : 0.f;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int64_t c = c0 + j, r = r0 + tx;
        if (c < t.C && r < t.R) t.B[c * t.ldb + r] = tile[tx][j];
    }
}

}  // namespace

hipError_t reduce_slices(const Dev& d, int64_t rows, int k, int64_t S, int nt, const float* partial,
                  float* out, int64_t ldo, bool trans) {
    const int64_t tot = rows * nt;
    hipLaunchKernelGGL(k_reduce_slices, dim3((unsigned)((tot + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, d.stream, rows, k, (int)S, nt, partial, out, ldo,
                       trans ? 1 : 0);
    return hipGetLastError();
}

size_t sweep_right_partial_floats(const Dev& d, int64_t R, int64_t C) {
    const RightPlan p16 = right_plan(d, R, C, 16), p32 = right_plan(d, R, C, 32);
    const int64_t S = p16.S > p32.S ? p16.S : p32.S;
    return S > 1 ? (size_t)(S * R * 32) : 0;
}

hipError_t sweep_right(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx, int k,
                       const float* A, int64_t lda, bool a_trans, float* Y, int64_t ldy,
                       float* partial) {
    if (R <= 0 || k <= 0 || C <= 0) return hipSuccess;
    // 16-byte vector loads of X (and of A^T) need aligned rows.
    const bool vec = ldx % 4 == 0 && aligned16(X) && (!a_trans || (lda % 4 == 0 && aligned16(A)));
    const RightPlan p = right_plan(d, R, C, k);
    dim3 grid((unsigned)p.tiles, (unsigned)p.S);
    const bool direct = p.S == 1;
    float* out = direct ? Y : partial;
    const int64_t ldo = direct ? ldy : p.nt;
#define LAUNCH_R(NT, SW, AT, D, V)                                                                  \
    hipLaunchKernelGGL((k_sweep_right<NT, SW, AT, D, V>), grid, dim3(kThreads), 0, d.stream, R, C, \
                       X, ldx, k, A, lda, out, ldo, p.span)
#define LAUNCH_R2(NT, SW, AT, D) \
    do { if (vec) LAUNCH_R(NT, SW, AT, D, true); else LAUNCH_R(NT, SW, AT, D, false); } while (0)
#define LAUNCH_R3(NT, SW)                                                                         \
    do {                                                                                          \
        if (a_trans) { if (direct) LAUNCH_R2(NT, SW, true, true); else LAUNCH_R2(NT, SW, true, false); } \
        else { if (direct) LAUNCH_R2(NT, SW, false, true); else LAUNCH_R2(NT, SW, false, false); }       \
    } while (0)
    if (p.nt == 16) { if (p.sw == 128) LAUNCH_R3(16, 128); else LAUNCH_R3(16, 256); }
    else { if (p.sw == 128) LAUNCH_R3(32, 128); else LAUNCH_R3(32, 256); }
#undef LAUNCH_R3
#undef LAUNCH_R2
#undef LAUNCH_R
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || direct) return e;
    return reduce_slices(d, R, k, p.S, p.nt, partial, Y, ldy, false);
}

size_t sweep_left_partial_floats(const Dev& d, int64_t R, int64_t C) {
    const LeftPlan p = left_plan(d, R, C, 32);
    return (size_t)(p.S * C * 32);
}

hipError_t sweep_left(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx, int k,
                      const float* B, int64_t ldb, float* Z, int64_t ldz, bool z_trans,
                      float* partial) {
    if (C <= 0 || k <= 0 || R <= 0) return hipSuccess;
    const bool vec = ldx % 4 == 0 && aligned16(X);
    const LeftPlan p = left_plan(d, R, C, k);
    dim3 grid((unsigned)p.tiles, (unsigned)p.S);
#define LAUNCH_L(NT, V)                                                                          \
    hipLaunchKernelGGL((k_sweep_left<NT, V>), grid, dim3(kThreads), 0, d.stream, R, C, X, ldx, k, \
                       B, ldb, partial, p.rspan)
    if (p.nt == 16) { if (vec) LAUNCH_L(16, true); else LAUNCH_L(16, false); }
    else { if (vec) LAUNCH_L(32, true); else LAUNCH_L(32, false); }
#undef LAUNCH_L
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce_slices(d, C, k, p.S, p.nt, partial, Z, ldz, z_trans);
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

namespace cnmf {

void sweep_desc_right(SweepDesc* s, int64_t R, int64_t C, const float* X, int64_t ldx, int k,
                      const float* AT, int64_t ldt, float* partial, float* Y, int64_t ldy) {
    *s = SweepDesc{};
    s->R = R;
    s->C = C;
    s->X = X;
    s->ldx = ldx;
    s->k = k;
    s->nt = k <= 16 ? 16 : 32;
    s->A = AT;
    s->lda = ldt;
    s->partial = partial;
    s->tiles = (int)((R + 31) / 32);
    s->S = 1;
    s->span = (C + 127) / 128 * 128;
    s->Y = Y;
    s->ldy = ldy;
    s->trans = 0;
}

void sweep_desc_left(SweepDesc* s, int64_t R, int64_t C, const float* X, int64_t ldx, int k,
                     const float* B, int64_t ldb, float* partial, float* Y, int64_t ldy,
                     bool trans) {
    *s = SweepDesc{};
    s->R = R;
    s->C = C;
    s->X = X;
    s->ldx = ldx;
    s->k = k;
    s->nt = k <= 16 ? 16 : 32;
    s->A = B;
    s->lda = ldb;
    s->partial = partial;
    s->tiles = (int)((C + 255) / 256);
    s->S = 1;
    s->span = (R + 15) / 16 * 16;
    s->Y = Y;
    s->ldy = ldy;
    s->trans = trans ? 1 : 0;
}

hipError_t sweep_right_batched(const Dev& d, const SweepDesc* desc, const WorkItem* work,
                               int64_t nwork) {
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sweep_right_batched, dim3((unsigned)nwork), dim3(kThreads), 0, d.stream,
                       desc, work);
    return hipGetLastError();
}

hipError_t sweep_left_batched(const Dev& d, const SweepDesc* desc, const WorkItem* work,
                              int64_t nwork) {
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sweep_left_batched, dim3((unsigned)nwork), dim3(kThreads), 0, d.stream,
                       desc, work);
    return hipGetLastError();
}

hipError_t reduce_batched(const Dev& d, const SweepDesc* desc, const WorkItem* work,
                          int64_t nwork, bool left) {
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_batched, dim3((unsigned)nwork), dim3(kThreads), 0, d.stream,
                       desc, work, left ? 1 : 0);
    return hipGetLastError();
}

hipError_t transpose_batched(const Dev& d, const TransDesc* desc, const WorkItem* work,
                             int64_t nwork) {
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose_batched, dim3((unsigned)nwork), dim3(kThreads), 0, d.stream,
                       desc, work);
    return hipGetLastError();
}

}  // namespace cnmf
