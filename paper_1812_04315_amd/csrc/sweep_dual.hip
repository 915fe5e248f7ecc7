// Dual X sweep: Y = X A and Z = X^T B from one read of X.  Every half-step
// of Algorithm 2 advances both chains, the n-space chain by a product with X
// and the m-space chain by a product with X^T, on panels that are already
// known; one pass over X serves both, so the randomized subspace iteration
// reads X 2q + 1 times instead of twice that.
//
// Workgroup = 256 columns of X times one slice of rows, streamed in stages
// of 32 rows x 256 columns through LDS (each wave loads 8 rows, one
// contiguous kilobyte per row and instruction; the next stage sits in
// registers while the current one is multiplied).  Both products are FP32
// MFMA with FP32 accumulation:
//   Z (left): wave w owns columns 64 w .. 64 w + 63 of the tile as two
//     32-column M tiles of v_mfma_f32_32x32x2f32 (M = column of X, K = row,
//     N = column of B) and accumulates over the whole row slice.
//   Y (right): wave w owns the 16 x 16 output tile rows 16 (w % 2) .. of the
//     stage, columns 16 (w / 2) .. of Y, on v_mfma_f32_16x16x4f32 with K =
//     the tile's 256 columns: lane group g = l / 16 takes columns 64 g + s
//     at MFMA s, whose A-panel values stay in registers for the whole launch.
//     Each stage's tile is a partial sum over this workgroup's 256 columns.
// Partials: Y over the C / 256 column tiles, Z over the row slices; two
// reductions sum them in a fixed order (bitwise reproducible results).
#include "internal.hpp"

namespace cnmf {

namespace {

constexpr int kThreads = 256;
constexpr int kDT = 256;       // columns of X per workgroup
constexpr int kDR = 32;        // rows of X per stage
constexpr int kDP = kDT + 4;   // LDS row pitch (floats): rows 4 banks apart

__device__ __forceinline__ v16f mfma32(float a, float b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of the 32x32 accumulator tile held in register r of lane l.
__device__ __forceinline__ int acc_row(int r, int lane) {
    return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// Keeps an MFMA result in vector registers at this point of the program
// (in the MFMA's own basic block, before any branch that reads it).
__device__ __forceinline__ void settle(v4f& acc) { asm volatile("" : "+v"(acc)); }

template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_sweep_dual(
    int64_t R, int64_t C, const float* __restrict__ X, int64_t ldx, int k,
    const float* __restrict__ AT, int64_t ldat, const float* __restrict__ B, int64_t ldb,
    float* __restrict__ part_y, float* __restrict__ part_z, int64_t rspan) {
    __shared__ __attribute__((aligned(16))) float xs[kDR * kDP];
    const int lane = threadIdx.x & 63;
    // wave-uniform (scalar registers): row addresses of X and B stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t c0 = (int64_t)blockIdx.x * kDT;
    const int64_t r_lo = (int64_t)blockIdx.y * rspan;
    const int64_t r_hi = min(R, r_lo + rspan);
    const int64_t nst = (r_hi - r_lo + kDR - 1) / kDR;
    const bool full = VEC && c0 + kDT <= C;   // uniform across the workgroup

    // left product: lane l is M row l % 32 (column of X), K index l / 32
    // (row of the stage), N column l % 32 of B (clamped: columns >= k of
    // the partial are never read)
    const int n32 = lane & 31, kl = lane >> 5;
    const int nb = n32 < k ? n32 : 0;
    // right product: output tile (mt, nt); lane l is M row l % 16, N column
    // l % 16, K group g = l / 16
    const int mt = wave & 1, nt = wave >> 1;
    const int n16 = lane & 15, g = lane >> 4;
    const int na = 16 * nt + n16;
    float ar[64];   // A[c0 + 64 g + s][na], zero past C or k
    {
        const int64_t cb = c0 + 64 * g;
        if (full && na < k) {
            const v4f* p = reinterpret_cast<const v4f*>(AT + na * ldat + cb);
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const v4f v = p[t];
#pragma unroll
                for (int u = 0; u < 4; ++u) ar[4 * t + u] = v[u];
            }
        } else {
#pragma unroll
            for (int s = 0; s < 64; ++s) {
                const int64_t c = cb + s;
                const bool in = na < k && c < C;
                const float v = AT[(in ? na : 0) * ldat + (c < C ? c : C - 1)];
                ar[s] = in ? v : 0.f;
            }
        }
    }

    v16f accL[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) accL[t][r] = 0.f;

    v4f xn[8];
    float bn[16], bc[16];
    int bn_valid = 0, bc_valid = 0;   // rows of the stage inside the slice
    // B rows 2 s + kl of a stage: a scalar row address (clamped to R - 1)
    // plus a per-lane offset; when the clamped row is the last one, lanes
    // kl = 1 read it too (their rows lie past the slice and are masked)
    const int64_t boff0 = nb, boff1 = (int64_t)kl * ldb + nb;
    auto load_b = [&](int64_t rb) {
        const int64_t nv = r_hi - rb;
        bn_valid = nv < kDR ? (int)nv : kDR;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int64_t row = rb + 2 * s;
            const int64_t base = row < R - 1 ? row : R - 1;
            bn[s] = B[base * ldb + (base < R - 1 ? boff1 : boff0)];
        }
    };
    auto load_fast = [&](int64_t st) {
        st = st < nst ? st : nst - 1;
        const int64_t rb = r_lo + kDR * st;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t row = rb + 8 * wave + i;
            const float* xr = X + (row < R ? row : R - 1) * ldx;
            xn[i] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(xr + c0 + 4 * lane));
        }
        load_b(rb);
    };
    auto load_slow = [&](int64_t st) {
        const int64_t rb = r_lo + kDR * st;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t row = rb + 8 * wave + i;
            const float* xr = X + (row < R ? row : R - 1) * ldx;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t c = c0 + 4 * lane + u;
                const float v = xr[c < C ? c : C - 1];
                xn[i][u] = c < C ? v : 0.f;
            }
        }
        load_b(rb);
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            *reinterpret_cast<v4f*>(&xs[(8 * wave + i) * kDP + 4 * lane]) = xn[i];
#pragma unroll
        for (int s = 0; s < 16; ++s) bc[s] = bn[s];
        bc_valid = bn_valid;
    };
    // both products of the stage in LDS; returns this wave's Y tile.  Step j
    // issues two left MFMAs (rows 2 j, 2 j + 1) and four right MFMAs
    // (columns 64 g + 4 j ..), three independent accumulation chains; the
    // LDS operands of step j + 1 are read while step j multiplies.
    auto compute = [&]() -> v4f {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        const float* xl = &xs[kl * kDP + 64 * wave + n32];
        const float* xr = &xs[(16 * mt + n16) * kDP + 64 * g];
        float l0 = xl[0], l1 = xl[32];
        v4f rv = *reinterpret_cast<const v4f*>(xr);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const float a0 = l0, a1 = l1;
            const v4f v = rv;
            if (j < 15) {
                l0 = xl[(2 * j + 2) * kDP];
                l1 = xl[(2 * j + 2) * kDP + 32];
                rv = *reinterpret_cast<const v4f*>(xr + 4 * j + 4);
            }
            const float bv = (2 * j + kl < bc_valid) ? bc[j] : 0.f;
            accL[0] = mfma32(a0, bv, accL[0]);
            accL[1] = mfma32(a1, bv, accL[1]);
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = mfma16(v[u], ar[4 * j + u], acc);
        }
        settle(acc);
        return acc;
    };
    // output layout of the 16x16 tile: register i of lane l is row 4 g + i,
    // column l % 16
    auto store_y = [&](int64_t rb, const v4f& y) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = rb + 16 * mt + 4 * g + i;
            if (row < r_hi) part_y[((int64_t)blockIdx.x * R + row) * 32 + na] = y[i];
        }
    };

    if (nst > 0 && full) {
        load_fast(0);
        store_stage();
        __syncthreads();
        for (int64_t st = 0; st < nst; ++st) {
            load_fast(st + 1);
            __builtin_amdgcn_sched_barrier(0);
            const v4f y = compute();
            __builtin_amdgcn_sched_barrier(0);
            store_y(r_lo + kDR * st, y);
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
            const v4f y = compute();
            store_y(r_lo + kDR * st, y);
        }
    }

#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t c = c0 + 64 * wave + 32 * t + acc_row(r, lane);
            if (c < C) part_z[((int64_t)blockIdx.y * C + c) * 32 + n32] = accL[t][r];
        }
}

bool al16(const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; }

int occ_dual() {
    static const int v = [] {
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &blocks, reinterpret_cast<const void*>(k_sweep_dual<true>), kThreads, 0) !=
                hipSuccess ||
            blocks < 1)
            blocks = 1;
        return blocks;
    }();
    return v;
}

struct DualPlan { int64_t tiles, S, rspan; };
DualPlan dual_plan(const Dev& d, int64_t R, int64_t C) {
    DualPlan p;
    p.tiles = (C + kDT - 1) / kDT;
    const int64_t stages = (R + kDR - 1) / kDR;
    p.S = pick_splits(p.tiles, stages, d.num_cus, occ_dual());
    p.rspan = kDR * ((stages + p.S - 1) / p.S);
    p.S = (R + p.rspan - 1) / p.rspan;
    return p;
}

}  // namespace

size_t sweep_dual_partial_floats(const Dev& d, int64_t R, int64_t C) {
    if (R <= 0 || C <= 0) return 0;
    const DualPlan p = dual_plan(d, R, C);
    return (size_t)(p.tiles * R + p.S * C) * 32;
}

hipError_t sweep_dual(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx, int k,
                      const float* AT, int64_t ldat, const float* B, int64_t ldb, float* Y,
                      int64_t ldy, float* Z, int64_t ldz, bool z_trans, float* partial) {
    if (R <= 0 || C <= 0 || k <= 0) return hipSuccess;
    if (k > 32) return hipErrorInvalidValue;
    // 16-byte vector loads of X and of the A panel need aligned rows.
    const bool vec = ldx % 4 == 0 && al16(X) && ldat % 4 == 0 && al16(AT);
    const DualPlan p = dual_plan(d, R, C);
    float* part_y = partial;
    float* part_z = partial + p.tiles * R * 32;
    dim3 grid((unsigned)p.tiles, (unsigned)p.S);
    if (vec)
        hipLaunchKernelGGL(k_sweep_dual<true>, grid, dim3(kThreads), 0, d.stream, R, C, X, ldx, k,
                           AT, ldat, B, ldb, part_y, part_z, p.rspan);
    else
        hipLaunchKernelGGL(k_sweep_dual<false>, grid, dim3(kThreads), 0, d.stream, R, C, X, ldx,
                           k, AT, ldat, B, ldb, part_y, part_z, p.rspan);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_slices(d, R, k, p.tiles, 32, part_y, Y, ldy, false);
    if (e != hipSuccess) return e;
    return reduce_slices(d, C, k, p.S, 32, part_z, Z, ldz, z_trans);
}

}  // namespace cnmf
