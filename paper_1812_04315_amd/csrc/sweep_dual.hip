// Dual X sweep: Y = X A and Z = X^T B from one read of X.  Every half-step
// of Algorithm 2 advances both chains, the n-space chain by a product with X
// and the m-space chain by a product with X^T, on panels that are already
// known; one pass over X serves both, so the randomized subspace iteration
// reads X 2q + 1 times instead of twice that.
#include "internal.hpp"

namespace cnmf {

namespace {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// Both products run on the BF16 matrix cores at FP32 accuracy.  Every
// FP32 operand is split exactly into three BF16 parts, x = h + m + l
// (h = bf16(x), m = bf16(x - h), l = x - h - m, all rounded to nearest
// even; l is exact because x - h - m keeps at most eight significant bits),
// and the six cross products with |term| >= 2^-16 |x a| are accumulated in
// FP32 (the "bf16x6" scheme of Henry, Tang and Heinecke, 2019): the dropped
// terms m a_l, l a_m, l a_l are below 2^-23 |x a|, the size of one FP32
// rounding.  v_mfma_f32_16x16x32_bf16 runs at sixteen times the FP32 rate,
// so six of them cost 3/8 of one FP32 product.
//
// Workgroup = 256 columns x one slice of rows, four waves side by side
// (wave w: columns 64 w .. 64 w + 63), groups of 32 rows.  Lane l (n = l %
// 16, g = l / 16) loads rows 4 t + g (t = 0..7) x columns 4 n .. 4 n + 3 of
// its wave's block (four 256-byte row pieces per instruction), so each lane
// holds eight rows of four columns:
//   Z (left) straight from registers: MFMA j (j = 0..3) takes column
//     4 n + j as M index n and rows 4 t + g as the K slots 8 g + t; the B
//     operand (rows x columns of B) comes pre-split in operand order.
//   Y (right) through LDS: the split parts are written row-major (each
//     lane pairs its own adjacent columns), read back as M = row, K = eight
//     consecutive columns; the A panel stays in registers, pre-split in
//     operand order.  The four waves' 32 x 32 tiles are summed in LDS in
//     wave order before one partial per workgroup is stored.
// Partials: Y over the C / 256 column tiles, Z over the row slices; two
// reductions sum them in a fixed order (bitwise reproducible results).
// ---------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

constexpr int kSW = 64;                     // columns per wave
constexpr int kST = 4 * kSW;                // columns per workgroup
constexpr int kSR = 32;                     // rows per group
constexpr int kSPitch = 2 * kSW + 16;       // bytes per row of a part in LDS
constexpr int kSPart = kSR * kSPitch;       // bytes per part
constexpr int kAWords = 4 * 2 * 2 * 3 * 256;   // pre-split A panel words per column tile
constexpr int kBWords = 3 * 2 * 256;           // pre-split B words per row group

// Two FP32 values -> one word of two BF16 (round to nearest even), first in
// the low half.
__device__ __forceinline__ unsigned pk_bf16(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((v2f){a, b}, v2bf));
}
__device__ __forceinline__ float lo_f(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_f(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

struct Split3 { unsigned h, m, l; };
__device__ __forceinline__ Split3 split3(float a, float b) {
    Split3 s;
    s.h = pk_bf16(a, b);
    a -= lo_f(s.h);
    b -= hi_f(s.h);
    s.m = pk_bf16(a, b);
    a -= lo_f(s.m);
    b -= hi_f(s.m);
    s.l = pk_bf16(a, b);
    return s;
}

__device__ __forceinline__ v4f mfma_sb(v4u a, v4u b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// The six cross terms (parts of x, parts of y), smallest first.  Callers
// take the term as the outer loop over several accumulators, so that
// consecutive matrix instructions never wait on each other's results.
__device__ constexpr int kTermX[6] = {2, 0, 1, 1, 0, 0};
__device__ constexpr int kTermY[6] = {0, 2, 1, 0, 1, 0};

// Operand-order split of the A panel (per column tile, wave, K step ks,
// N tile nt, part, lane, word: columns 64 w + 32 ks + 8 (l / 16) + 2 d, + 1
// of the tile, N column 16 nt + l % 16) and of B (per row group, part, N
// tile, lane, word: rows 4 (2 d) + l / 16, 4 (2 d + 1) + l / 16 of the group,
// N column 16 nt + l % 16); zero outside the operands.
__global__ __launch_bounds__(kThreads) void k_split_operands(
    int64_t R, int64_t C, int k, const float* __restrict__ AT, int64_t ldat,
    const float* __restrict__ B, int64_t ldb, unsigned* __restrict__ ap, unsigned* __restrict__ bp,
    int64_t a_items, int64_t items) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= items) return;
    const int lane = (int)(e >> 2) & 63, d = (int)e & 3;
    const int nc = lane & 15, g = lane >> 4;
    if (e < a_items) {
        // e = ((((T * 4 + w) * 2 + ks) * 2 + nt) * 256 + lane * 4 + d)
        const int64_t u = e >> 8;
        const int nt = (int)(u & 1), ks = (int)((u >> 1) & 1);
        const int64_t tw = u >> 2;   // T * 4 + w
        const int cn = 16 * nt + nc;
        const int64_t c = tw * kSW + 32 * ks + 8 * g + 2 * d;
        const float a0 = (cn < k && c < C) ? AT[cn * ldat + c] : 0.f;
        const float a1 = (cn < k && c + 1 < C) ? AT[cn * ldat + c + 1] : 0.f;
        const Split3 s = split3(a0, a1);
        unsigned* o = ap + u * (3 * 256) + lane * 4 + d;
        o[0] = s.h;
        o[256] = s.m;
        o[512] = s.l;
        return;
    }
    const int64_t f = e - a_items;
    // f = (G * 2 + nt) * 256 + lane * 4 + d
    const int64_t u = f >> 8;
    const int nt = (int)(u & 1);
    const int64_t G = u >> 1;
    const int cn = 16 * nt + nc;
    const int64_t r0 = kSR * G + 4 * (2 * d) + g, r1 = r0 + 4;
    const float b0 = (cn < k && r0 < R) ? B[r0 * ldb + cn] : 0.f;
    const float b1 = (cn < k && r1 < R) ? B[r1 * ldb + cn] : 0.f;
    const Split3 s = split3(b0, b1);
    unsigned* o = bp + (G * 3 * 2 + nt) * 256 + lane * 4 + d;
    o[0] = s.h;
    o[2 * 256] = s.m;
    o[4 * 256] = s.l;
}

// WIDE: 64-bit lane offsets (row pitches of 2^25 floats and more).  Rows
// that are not 16-byte aligned (VEC false) take clamped scalar loads, whose
// addresses need more registers: one workgroup per CU there.
template <bool VEC, bool WIDE>
__global__ __launch_bounds__(kThreads, VEC ? 2 : 1) void k_sweep_dual_sb(
    int64_t R, int64_t C, const float* __restrict__ X, int64_t ldx,
    const unsigned* __restrict__ ap, const unsigned* __restrict__ bp,
    float* __restrict__ part_y, float* __restrict__ part_z, int64_t rspan) {
    __shared__ __attribute__((aligned(16))) unsigned char xs[4][3][kSPart];
    __shared__ __attribute__((aligned(16))) float ys[4][kSR][36];   // rows 16 banks apart
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = lane & 15, g = lane >> 4;
    const int64_t T = blockIdx.x;
    const int64_t cw = T * kST + (int64_t)wave * kSW;   // first column of this wave
    const int64_t r_lo = (int64_t)blockIdx.y * rspan;
    const int64_t r_hi = min(R, r_lo + rspan);
    const int64_t ngr = (r_hi - r_lo + kSR - 1) / kSR;
    const bool full = VEC && cw + kSW <= C;   // uniform across the wave

    // A panel, pre-split: [ks][nt][part]
    v4u pa[2][2][3];
    {
        const v4u* q = reinterpret_cast<const v4u*>(ap) + (T * 4 + wave) * (2 * 2 * 3 * 64) + lane;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int h = 0; h < 3; ++h) pa[ks][nt][h] = q[((ks * 2 + nt) * 3 + h) * 64];
    }
    v4f zacc[4][2];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) zacc[j][nt] = v4f{0.f, 0.f, 0.f, 0.f};

    const int64_t cl = cw + 4 * n;
    // groups with all 32 rows inside the slice and X: straight-line 16-byte
    // loads from a wave-uniform row base plus 32-bit lane offsets
    const int64_t nfull = full ? (r_hi - r_lo) / kSR : 0;
    using Ofs = typename std::conditional<WIDE, int64_t, int>::type;
    const Ofs lofs = (Ofs)(g * ldx + 4 * n);
    auto load_x = [&](int64_t gi, v4f (&xv)[8]) {
        const int64_t rb = r_lo + kSR * gi;
        if (gi < nfull) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float* xg = X + (rb + 4 * t) * ldx + cw;   // wave-uniform
                xv[t] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(xg + lofs));
            }
        } else {
            // ragged: rows and columns clamped into X (their B and A parts
            // are zero)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int64_t row = rb + 4 * t + g;
                const float* xr = X + (row < R ? row : R - 1) * ldx;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t c = cl + u;
                    xv[t][u] = xr[c < C ? c : C - 1];
                }
            }
        }
    };
    auto load_b = [&](int64_t gi, v4u (&bv)[3][2]) {
        const int64_t grp = (r_lo + kSR * gi) / kSR;
        const v4u* q = reinterpret_cast<const v4u*>(bp) + grp * (3 * 2 * 64) + lane;
#pragma unroll
        for (int h = 0; h < 3; ++h)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) bv[h][nt] = q[(h * 2 + nt) * 64];
    };

    unsigned char* myx = &xs[wave][0][0];
    v4f xv[8];
    v4u bv[3][2];
    if (ngr > 0) {
        load_x(0, xv);
        load_b(0, bv);
    }
    // Each group's loads are issued into the registers of the group before
    // as soon as those are consumed (X after the split, B after the left
    // products), a whole step ahead of their use; two workgroups per CU
    // overlap one's matrix work with the other's vector work.
    for (int64_t gi = 0; gi < ngr; ++gi) {
        const int64_t gn = gi + 1 < ngr ? gi + 1 : gi;
        // columns in two halves (registers): split, left products, right
        // operand to LDS
#pragma unroll
        for (int jh = 0; jh < 2; ++jh) {
            // split: P[jj][part] word d = rows (2 d, 2 d + 1) of column 2 jh + jj
            v4u P[2][3];
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const Split3 sp = split3(xv[2 * d][2 * jh + jj], xv[2 * d + 1][2 * jh + jj]);
                    P[jj][0][d] = sp.h;
                    P[jj][1][d] = sp.m;
                    P[jj][2][d] = sp.l;
                }
            if (jh == 1) {
                // X of this group consumed: the next group's rows go in
                __builtin_amdgcn_sched_barrier(0);
                load_x(gn, xv);
                __builtin_amdgcn_sched_barrier(0);
            }
            // left: Z[col 4 n + j][16 nt + .] += X^T B over the group's rows
#pragma unroll
            for (int e = 0; e < 6; ++e)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
                        zacc[2 * jh + jj][nt] =
                            mfma_sb(P[jj][kTermX[e]], bv[kTermY[e]][nt], zacc[2 * jh + jj][nt]);
            if (jh == 1) {
                __builtin_amdgcn_sched_barrier(0);
                load_b(gn, bv);
                __builtin_amdgcn_sched_barrier(0);
            }
            // right operand: row 4 t + g, columns 4 n + 2 jh, + 1 as one word
            // per part
#pragma unroll
            for (int h = 0; h < 3; ++h)
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const unsigned w0 = P[0][h][t >> 1], w1 = P[1][h][t >> 1];
                    const unsigned v = (t & 1) ? ((w0 >> 16) | (w1 & 0xffff0000u))
                                               : ((w0 & 0xffffu) | (w1 << 16));
                    *reinterpret_cast<unsigned*>(myx + h * kSPart + (4 * t + g) * kSPitch + 8 * n +
                                                 4 * jh) = v;
                }
        }
        // right: Y[row 16 mt + .][16 nt + .] over the wave's 64 columns
        v4f yacc[2][2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) yacc[mt][nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                v4u xa[3];
#pragma unroll
                for (int h = 0; h < 3; ++h)
                    xa[h] = *reinterpret_cast<const v4u*>(
                        myx + h * kSPart + (16 * mt + n) * kSPitch + 2 * (32 * ks + 8 * g));
#pragma unroll
                for (int e = 0; e < 6; ++e)
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
                        yacc[mt][nt] = mfma_sb(xa[kTermX[e]], pa[ks][nt][kTermY[e]], yacc[mt][nt]);
            }
        // the four waves' tiles summed in wave order, this workgroup's
        // partial stored; the first barrier keeps the previous group's
        // readers ahead of these writes
        lds_barrier();
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) ys[wave][16 * mt + 4 * g + i][16 * nt + n] = yacc[mt][nt][i];
        lds_barrier();
        const int rr = 8 * wave + (lane >> 3), cc = 4 * (lane & 7);
        v4f sum = *reinterpret_cast<const v4f*>(&ys[0][rr][cc]);
#pragma unroll
        for (int w = 1; w < 4; ++w) sum += *reinterpret_cast<const v4f*>(&ys[w][rr][cc]);
        const int64_t row = r_lo + kSR * gi + rr;
        if (row < r_hi) *reinterpret_cast<v4f*>(&part_y[(T * R + row) * 32 + cc]) = sum;
    }

    // Z partial of this slice: lane holds column 16 g + 4 i + j, N 16 nt + n
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t c = cw + 16 * g + 4 * i + j;
                if (c < C) part_z[((int64_t)blockIdx.y * C + c) * 32 + 16 * nt + n] = zacc[j][nt][i];
            }
}

// ---------------------------------------------------------------------------
// BF16 form of the dual pass: X holds bfloat16 bit patterns and both
// skinny operands are rounded to bfloat16 (nearest even), FP32 accumulation
// on v_mfma_f32_16x16x32_bf16 -- the products of the one-sided BF16 sweeps,
// from one read of X.  Same organisation as the kernel above with one part
// per operand; a lane's sixteen bytes of a row are eight columns, so a wave
// takes 128 columns and a workgroup 512:
//   Z: MFMA j (j = 0..7) takes column 8 n + j as M index n; its K words
//     pair rows 4 (2 d) + g and 4 (2 d + 1) + g, repacked from the loaded
//     rows by one permute per word.
//   Y: the loaded rows go to LDS unchanged and come back as M = row,
//     K = eight consecutive columns.
// ---------------------------------------------------------------------------
constexpr int kBW = 128;                    // columns per wave
constexpr int kBT = 4 * kBW;                // columns per workgroup
constexpr int kBPitch = 2 * kBW + 16;       // bytes per LDS row
constexpr int kBAWords = 4 * 4 * 2 * 256;   // rounded A panel words per column tile
constexpr int kBBWords = 2 * 256;           // rounded B words per row group

// Operand-order rounding of the A panel (per column tile, wave, K step ks,
// N tile nt, lane, word: columns 128 w + 32 ks + 8 (l / 16) + 2 d, + 1 of
// the tile) and of B (per row group, N tile, lane, word: rows 8 d + l / 16,
// 8 d + 4 + l / 16 of the group); N column 16 nt + l % 16; zero outside.
__global__ __launch_bounds__(kThreads) void k_round_operands(
    int64_t R, int64_t C, int k, const float* __restrict__ AT, int64_t ldat,
    const float* __restrict__ B, int64_t ldb, unsigned* __restrict__ ap, unsigned* __restrict__ bp,
    int64_t a_items, int64_t items) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= items) return;
    const int lane = (int)(e >> 2) & 63, d = (int)e & 3;
    const int nc = lane & 15, g = lane >> 4;
    if (e < a_items) {
        // e = (((T * 4 + w) * 4 + ks) * 2 + nt) * 256 + lane * 4 + d
        const int64_t u = e >> 8;
        const int nt = (int)(u & 1), ks = (int)((u >> 1) & 3);
        const int64_t tw = u >> 3;   // T * 4 + w
        const int cn = 16 * nt + nc;
        const int64_t c = tw * kBW + 32 * ks + 8 * g + 2 * d;
        const float a0 = (cn < k && c < C) ? AT[cn * ldat + c] : 0.f;
        const float a1 = (cn < k && c + 1 < C) ? AT[cn * ldat + c + 1] : 0.f;
        ap[e] = pk_bf16(a0, a1);
        return;
    }
    const int64_t f = e - a_items;
    // f = (G * 2 + nt) * 256 + lane * 4 + d
    const int nt = (int)((f >> 8) & 1);
    const int64_t G = f >> 9;
    const int cn = 16 * nt + nc;
    const int64_t r0 = kSR * G + 8 * d + g, r1 = r0 + 4;
    const float b0 = (cn < k && r0 < R) ? B[r0 * ldb + cn] : 0.f;
    const float b1 = (cn < k && r1 < R) ? B[r1 * ldb + cn] : 0.f;
    bp[f] = pk_bf16(b0, b1);
}

template <bool VEC, bool WIDE>
__global__ __launch_bounds__(kThreads, 2) void k_sweep_dual_bf16(
    int64_t R, int64_t C, const uint16_t* __restrict__ X, int64_t ldx,
    const unsigned* __restrict__ ap, const unsigned* __restrict__ bp,
    float* __restrict__ part_y, float* __restrict__ part_z, int64_t rspan) {
    __shared__ __attribute__((aligned(16))) unsigned char xs[4][kSR * kBPitch];
    __shared__ __attribute__((aligned(16))) float ys[4][kSR][36];   // rows 16 banks apart
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = lane & 15, g = lane >> 4;
    const int64_t T = blockIdx.x;
    const int64_t cw = T * kBT + (int64_t)wave * kBW;   // first column of this wave
    const int64_t r_lo = (int64_t)blockIdx.y * rspan;
    const int64_t r_hi = min(R, r_lo + rspan);
    const int64_t ngr = (r_hi - r_lo + kSR - 1) / kSR;
    const bool full = VEC && cw + kBW <= C;   // uniform across the wave

    // A panel, rounded: [ks][nt]
    v4u pa[4][2];
    {
        const v4u* q = reinterpret_cast<const v4u*>(ap) + (T * 4 + wave) * (4 * 2 * 64) + lane;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) pa[ks][nt] = q[(ks * 2 + nt) * 64];
    }
    v4f zacc[8][2];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) zacc[j][nt] = v4f{0.f, 0.f, 0.f, 0.f};

    const int64_t cl = cw + 8 * n;
    const int64_t nfull = full ? (r_hi - r_lo) / kSR : 0;
    using Ofs = typename std::conditional<WIDE, int64_t, int>::type;
    const Ofs lofs = (Ofs)(g * ldx + 8 * n);
    // groups with all 32 rows inside the slice and X: 16-byte loads from a
    // wave-uniform row base plus a lane offset
    auto load_fast = [&](int64_t gi, v4u (&xv)[8]) {
        const int64_t rb = r_lo + kSR * gi;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const uint16_t* xg = X + (rb + 4 * t) * ldx + cw;   // wave-uniform
            xv[t] = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(xg + lofs));
        }
    };
    // ragged: rows and columns clamped into X (their B and A values are zero)
    auto load_slow = [&](int64_t gi, v4u (&xv)[8]) {
        const int64_t rb = r_lo + kSR * gi;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int64_t row = rb + 4 * t + g;
            const uint16_t* xr = X + (row < R ? row : R - 1) * ldx;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t c0 = cl + 2 * u, c1 = c0 + 1;
                const unsigned lo = xr[c0 < C ? c0 : C - 1];
                const unsigned hi = xr[c1 < C ? c1 : C - 1];
                xv[t][u] = lo | (hi << 16);
            }
        }
    };
    auto load_b = [&](int64_t gi, v4u (&bv)[2]) {
        const int64_t grp = (r_lo + kSR * gi) / kSR;
        const v4u* q = reinterpret_cast<const v4u*>(bp) + grp * (2 * 64) + lane;
        bv[0] = q[0];
        bv[1] = q[64];
    };

    unsigned char* myx = &xs[wave][0];
    v4u xv[8];
    v4u bv[2];
    // one group; PREFETCH: the next full group's rows and B values are
    // issued as soon as this group's are consumed, a step ahead of their use
    auto step = [&](int64_t gi, auto prefetch) {
        constexpr bool PREFETCH = decltype(prefetch)::value;
        // rows to LDS unchanged (row 4 t + g, columns 8 n .. 8 n + 7)
#pragma unroll
        for (int t = 0; t < 8; ++t)
            *reinterpret_cast<v4u*>(myx + (4 * t + g) * kBPitch + 16 * n) = xv[t];
        // left: K words of column 8 n + j pair rows 8 d + g and 8 d + 4 + g
        v4u P[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const unsigned w0 = xv[2 * d][j >> 1], w1 = xv[2 * d + 1][j >> 1];
                P[j][d] = (j & 1) ? ((w0 >> 16) | (w1 & 0xffff0000u)) : ((w0 & 0xffffu) | (w1 << 16));
            }
        if constexpr (PREFETCH) {
            __builtin_amdgcn_sched_barrier(0);
            load_fast(gi + 1 < nfull ? gi + 1 : gi, xv);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) zacc[j][nt] = mfma_sb(P[j], bv[nt], zacc[j][nt]);
        if constexpr (PREFETCH) {
            __builtin_amdgcn_sched_barrier(0);
            load_b(gi + 1 < ngr ? gi + 1 : gi, bv);
            __builtin_amdgcn_sched_barrier(0);
        }
        // right: Y[row 16 mt + .][16 nt + .] over the wave's 128 columns
        v4f yacc[2][2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) yacc[mt][nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const v4u xa = *reinterpret_cast<const v4u*>(myx + (16 * mt + n) * kBPitch +
                                                             2 * (32 * ks + 8 * g));
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) yacc[mt][nt] = mfma_sb(xa, pa[ks][nt], yacc[mt][nt]);
            }
        // the four waves' tiles summed in wave order, this workgroup's
        // partial stored; the first barrier keeps the previous group's
        // readers ahead of these writes
        lds_barrier();
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) ys[wave][16 * mt + 4 * g + i][16 * nt + n] = yacc[mt][nt][i];
        lds_barrier();
        const int rr = 8 * wave + (lane >> 3), cc = 4 * (lane & 7);
        v4f sum = *reinterpret_cast<const v4f*>(&ys[0][rr][cc]);
#pragma unroll
        for (int w = 1; w < 4; ++w) sum += *reinterpret_cast<const v4f*>(&ys[w][rr][cc]);
        const int64_t row = r_lo + kSR * gi + rr;
        if (row < r_hi) *reinterpret_cast<v4f*>(&part_y[(T * R + row) * 32 + cc]) = sum;
    };
    // every wave runs ngr steps (two barriers each), whichever path it takes
    int64_t gi = 0;
    if (nfull > 0) {
        load_fast(0, xv);
        load_b(0, bv);
        for (; gi < nfull; ++gi) step(gi, std::true_type{});
    }
    for (; gi < ngr; ++gi) {
        load_slow(gi, xv);
        load_b(gi, bv);
        step(gi, std::false_type{});
    }

    // Z partial of this slice: lane holds column 32 g + 8 i + j, N 16 nt + n
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t c = cw + 32 * g + 8 * i + j;
                if (c < C) part_z[((int64_t)blockIdx.y * C + c) * 32 + 16 * nt + n] = zacc[j][nt][i];
            }
}

bool al16(const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; }

struct DualPlan { int64_t tiles, S, rspan; };

// two workgroups per CU, slices a whole number of groups
DualPlan dual_plan(const Dev& d, int64_t R, int64_t C) {
    DualPlan p;
    p.tiles = (C + kST - 1) / kST;
    const int64_t groups = (R + kSR - 1) / kSR;
    p.S = pick_splits(p.tiles, groups, d.num_cus, 2);
    p.rspan = kSR * ((groups + p.S - 1) / p.S);
    p.S = (R + p.rspan - 1) / p.rspan;
    return p;
}

template <bool VEC, bool WIDE>
void launch_dual(const Dev& d, dim3 grid, int64_t R, int64_t C, const float* X, int64_t ldx,
                 const unsigned* ap, const unsigned* bp, float* part_y, float* part_z,
                 int64_t rspan) {
    hipLaunchKernelGGL((k_sweep_dual_sb<VEC, WIDE>), grid, dim3(kThreads), 0, d.stream, R, C, X,
                       ldx, ap, bp, part_y, part_z, rspan);
}

DualPlan bf_plan(const Dev& d, int64_t R, int64_t C) {
    DualPlan p;
    p.tiles = (C + kBT - 1) / kBT;
    const int64_t groups = (R + kSR - 1) / kSR;
    p.S = pick_splits(p.tiles, groups, d.num_cus, 2);
    p.rspan = kSR * ((groups + p.S - 1) / p.S);
    p.S = (R + p.rspan - 1) / p.rspan;
    return p;
}

template <bool VEC, bool WIDE>
void launch_dual_bf16(const Dev& d, dim3 grid, int64_t R, int64_t C, const uint16_t* X,
                      int64_t ldx, const unsigned* ap, const unsigned* bp, float* part_y,
                      float* part_z, int64_t rspan) {
    hipLaunchKernelGGL((k_sweep_dual_bf16<VEC, WIDE>), grid, dim3(kThreads), 0, d.stream, R, C,
                       X, ldx, ap, bp, part_y, part_z, rspan);
}

}  // namespace

size_t sweep_dual_bf16_partial_floats(const Dev& d, int64_t R, int64_t C) {
    if (R <= 0 || C <= 0) return 0;
    const DualPlan p = bf_plan(d, R, C);
    return (size_t)(p.tiles * R + p.S * C) * 32 + (size_t)p.tiles * kBAWords +
           (size_t)((R + kSR - 1) / kSR) * kBBWords;
}

hipError_t sweep_dual_bf16(const Dev& d, int64_t R, int64_t C, const uint16_t* Xb, int64_t ldx,
                           int k, const float* AT, int64_t ldat, const float* B, int64_t ldb,
                           float* Y, int64_t ldy, float* Z, int64_t ldz, bool z_trans,
                           float* partial) {
    if (R <= 0 || C <= 0 || k <= 0) return hipSuccess;
    if (k > 32) return hipErrorInvalidValue;
    const bool vec = ldx % 8 == 0 && al16(Xb);
    const bool wide = kSR * ldx >= ((int64_t)1 << 30);
    const DualPlan p = bf_plan(d, R, C);
    float* part_y = partial;
    float* part_z = partial + p.tiles * R * 32;
    unsigned* ap = reinterpret_cast<unsigned*>(part_z + p.S * C * 32);
    unsigned* bp = ap + p.tiles * kBAWords;
    const int64_t a_items = p.tiles * kBAWords;
    const int64_t items = a_items + ((R + kSR - 1) / kSR) * kBBWords;
    hipLaunchKernelGGL(k_round_operands, dim3((unsigned)((items + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, d.stream, R, C, k, AT, ldat, B, ldb, ap, bp, a_items,
                       items);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)p.tiles, (unsigned)p.S);
    if (vec && !wide)
        launch_dual_bf16<true, false>(d, grid, R, C, Xb, ldx, ap, bp, part_y, part_z, p.rspan);
    else if (vec)
        launch_dual_bf16<true, true>(d, grid, R, C, Xb, ldx, ap, bp, part_y, part_z, p.rspan);
    else
        launch_dual_bf16<false, true>(d, grid, R, C, Xb, ldx, ap, bp, part_y, part_z, p.rspan);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_slices(d, R, k, p.tiles, 32, part_y, Y, ldy, false);
    if (e != hipSuccess) return e;
    return reduce_slices(d, C, k, p.S, 32, part_z, Z, ldz, z_trans);
}

size_t sweep_dual_partial_floats(const Dev& d, int64_t R, int64_t C) {
    if (R <= 0 || C <= 0) return 0;
    const DualPlan p = dual_plan(d, R, C);
    return (size_t)(p.tiles * R + p.S * C) * 32 + (size_t)p.tiles * kAWords +
           (size_t)((R + kSR - 1) / kSR) * kBWords;
}

hipError_t sweep_dual(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx, int k,
                      const float* AT, int64_t ldat, const float* B, int64_t ldb, float* Y,
                      int64_t ldy, float* Z, int64_t ldz, bool z_trans, float* partial) {
    if (R <= 0 || C <= 0 || k <= 0) return hipSuccess;
    if (k > 32) return hipErrorInvalidValue;
    // 16-byte vector loads of X need aligned rows
    const bool vec = ldx % 4 == 0 && al16(X);
    // lane offsets within a 32-row group fit 32 bits below this pitch
    const bool wide = kSR * ldx >= ((int64_t)1 << 30);
    const DualPlan p = dual_plan(d, R, C);
    float* part_y = partial;
    float* part_z = partial + p.tiles * R * 32;
    unsigned* ap = reinterpret_cast<unsigned*>(part_z + p.S * C * 32);
    unsigned* bp = ap + p.tiles * kAWords;
    const int64_t a_items = p.tiles * (kAWords / 3);
    const int64_t items = a_items + ((R + kSR - 1) / kSR) * (kBWords / 3);
    hipLaunchKernelGGL(k_split_operands, dim3((unsigned)((items + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, d.stream, R, C, k, AT, ldat, B, ldb, ap, bp, a_items,
                       items);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)p.tiles, (unsigned)p.S);
    if (vec && !wide)
        launch_dual<true, false>(d, grid, R, C, X, ldx, ap, bp, part_y, part_z, p.rspan);
    else if (vec)
        launch_dual<true, true>(d, grid, R, C, X, ldx, ap, bp, part_y, part_z, p.rspan);
    else
        launch_dual<false, true>(d, grid, R, C, X, ldx, ap, bp, part_y, part_z, p.rspan);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = reduce_slices(d, R, k, p.tiles, 32, part_y, Y, ldy, false);
    if (e != hipSuccess) return e;
    return reduce_slices(d, C, k, p.S, 32, part_z, Z, ldz, z_trans);
}

}  // namespace cnmf
