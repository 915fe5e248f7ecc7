// Orthonormal bases for randomized subspace iteration (Sec. 3, Algorithm 2:
// "QR decomposition", "orthonormal bases" of each sketch and half-step).
//
// CholeskyQR on an N x l FP32 panel (l <= 32), one persistent launch:
//   pass 1: W = Y^T Y in FP64, right-looking Cholesky with the numerical-
//           rank rule; if a column is deficient, the same on the augmented
//           W = [Y P]^T [Y P] (P = replacement pool) with the swaps;
//           Q1 = Y^ R^-1 (FP64 arithmetic) where Y^ is Y with deficient
//           columns swapped for pool columns;
//   pass 2 (only for an ill-conditioned panel, see below): W = Q1^T Q1,
//           Cholesky, Q = Q1 R2^-1 (CholeskyQR2).
// The FP64 Gram of FP32 data has exact products, and CholeskyQR loses
// orthogonality in proportion to eps cond^2 in the precision of its Gram and
// factorisation, here FP64, where cond is that of Y with unit columns, about
// 1 / sqrt(min_j pivot_j / W_jj).  While min_j pivot_j / W_jj >= 1e-7 that
// loss is below 1e-9, under the FP32 rounding of Q itself, and a second
// pass would only repeat that rounding: Q = Q1.  Otherwise (and after
// column replacements) pass 2 follows.
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

#include <algorithm>

namespace cnmf {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxW = 64;        // augmented width 2 l
constexpr int kMaxPairs = kOrthMaxPairs;   // pairs of a 64-column Gram
constexpr int kPairsPerThread = (kMaxPairs + kThreads - 1) / kThreads;   // 9
constexpr int kTile = 32;
constexpr int kGramBlocksPerWave = 3;   // ceil(10 upper 16 x 16 blocks of a 64-column Gram / 4 waves)
constexpr double kPolish = 1e-7;   // min pivot ratio below which pass 2 runs

// accumulator of one 16 x 16 FP64 matrix-core product: register i of lane t
// holds row 4 i + t / 16, column t mod 16
typedef double v4d __attribute__((ext_vector_type(4)));

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

// Pair e of the upper triangle of a w x w matrix in row order (row a holds
// (a, a) .. (a, w - 1)): counted from the end, f = T - 1 - e lies in the
// k-th row from the bottom, k (k + 1) / 2 <= f < (k + 1) (k + 2) / 2.
__device__ __forceinline__ void pair_of(int e, int w, int* a, int* b) {
    const int T = w * (w + 1) / 2;
    const int f = T - 1 - e;
    int k = (int)((sqrtf(8.f * (float)f + 1.f) - 1.f) * 0.5f);
    if ((k + 1) * (k + 2) / 2 <= f) ++k;   // float rounding, one step either way
    if (k * (k + 1) / 2 > f) --k;
    *a = w - 1 - k;
    *b = w - 1 - (f - k * (k + 1) / 2);
}

struct Shared {
    double M[kMaxW][kMaxW + 1];
    double tile[kTile][kMaxW + 1];
    double Ri[32][33];
    double rvec[kMaxW];
    double dinv[32];
    double ref[kMaxW];
    double minrat;   // min_j pivot_j / W_jj of the last factorisation
    int sel[32];
    int flag;
    int timeout;
};

// (row, column) of element e = threadIdx.x + kThreads q of a row-major tile
// with w columns, without a division per element: stepping e by
// kThreads = A w + B moves A rows and B columns, with at most one carry.
template <int N>
__device__ __forceinline__ void tile_coords(int w, int (&er)[N], int (&ec)[N]) {
    const int A = kThreads / w, B = kThreads - A * w;
    int rr = (int)threadIdx.x / w, c = (int)threadIdx.x - rr * w;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        er[q] = rr;
        ec[q] = c;
        c += B;
        rr += A;
        if (c >= w) {
            c -= w;
            ++rr;
        }
    }
}

}  // namespace


namespace {

// Gram partial over this workgroup's rows: pairs (a <= b) of the w columns of
// [A | P] (w = l: only A).  A element (r, c) at A[r * l + c].
// Tiles of 32 rows are staged in LDS as FP64 (the next tile's loads in flight
// while the current one is multiplied).  The Gram's upper 16 x 16 blocks
// (at most 10 for w <= 64) go round-robin to the four waves, each a tile^T
// tile product on the FP64 matrix cores, K = rows in steps of 4.  At the end
// the blocks pass through sh.M into the per-thread pair accumulators.
__device__ void gram_partial(const OrthArgs& g, Shared& sh, const float* A, int w, int64_t r0,
                             int64_t r1, double (&acc)[kPairsPerThread], int (&pa)[kPairsPerThread],
                             int (&pb)[kPairsPerThread]) {
    const int l = g.l;
    // each thread's elements of a tile (kTile * w <= 8 * kThreads); the first
    // tile's loads go out before the index set-up below
    constexpr int kPer = (kTile * kMaxW + kThreads - 1) / kThreads;
    float vn[kPer];
    int er[kPer], ec[kPer];
    tile_coords(w, er, ec);
    auto load_tile = [&](int64_t t0) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int rr = er[q], c = ec[q];
            const int64_t r = t0 + rr;
            float v = 0.f;
            if (rr < kTile && r < r1)
                v = (c < l) ? A[r * l + c] : g.P[r * g.p_rs + (c - l) * g.p_cs];
            vn[q] = v;
        }
    };
    if (r0 < r1) load_tile(r0);
    const int npairs = w * (w + 1) / 2;
#pragma unroll
    for (int s = 0; s < kPairsPerThread; ++s) {
        const int e = threadIdx.x + s * kThreads;
        int a = 0, b = -1;
        if (e < npairs) pair_of(e, w, &a, &b);
        pa[s] = a;
        pb[s] = b;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // this wave's blocks (at, bt), at <= bt < nb, counted in row order
    const int nb = (w + 15) >> 4, nblocks = nb * (nb + 1) / 2;
    int bat[kGramBlocksPerWave], bbt[kGramBlocksPerWave];
#pragma unroll
    for (int u = 0; u < kGramBlocksPerWave; ++u) {
        int j = wave + 4 * u, at = 0;
        while (at < nb && j >= nb - at) { j -= nb - at; ++at; }
        bat[u] = at;
        bbt[u] = at + j;   // valid when wave + 4 u < nblocks
    }
    v4d gacc[kGramBlocksPerWave];
#pragma unroll
    for (int u = 0; u < kGramBlocksPerWave; ++u) gacc[u] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        lds_barrier();   // every wave is done with the previous tile
#pragma unroll
        for (int q = 0; q < kPer; ++q)
            if (er[q] < kTile) sh.tile[er[q]][ec[q]] = (double)vn[q];
        if (t0 + kTile < r1) load_tile(t0 + kTile);
        lds_barrier();   // LDS only: the loads above stay in flight
#pragma unroll
        for (int u = 0; u < kGramBlocksPerWave; ++u) {
            if (wave + 4 * u < nblocks) {
                const int ca = 16 * bat[u] + li, cb = 16 * bbt[u] + li;
#pragma unroll
                for (int s = 0; s < kTile / 4; ++s) {
                    const int rr = 4 * s + lk;
                    const double x = ca < w ? sh.tile[rr][ca] : 0.0;
                    const double y = cb < w ? sh.tile[rr][cb] : 0.0;
                    gacc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, gacc[u], 0, 0, 0);
                }
            }
        }
    }
    // block element (4 i + lk, li) of register i -> sh.M, then the pairs
#pragma unroll
    for (int u = 0; u < kGramBlocksPerWave; ++u) {
        if (wave + 4 * u < nblocks) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sh.M[16 * bat[u] + 4 * i + lk][16 * bbt[u] + li] = gacc[u][i];
        }
    }
    lds_barrier();
#pragma unroll
    for (int s = 0; s < kPairsPerThread; ++s) acc[s] = pb[s] >= 0 ? sh.M[pa[s]][pb[s]] : 0.0;
}

// Sum of the partial Grams over the grid -> sh.M (full symmetric, w x w).
// Returns false on a stalled exchange.
__device__ bool gram_exchange(const OrthArgs& g, Shared& sh, int w, unsigned tag_part,
                              unsigned tag_red, const double (&acc)[kPairsPerThread],
                              const int (&pa)[kPairsPerThread], const int (&pb)[kPairsPerThread],
                              const unsigned blk, const unsigned nblk) {
    const int npairs = w * (w + 1) / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // 1. publish this workgroup's partial
#pragma unroll
    for (int s = 0; s < kPairsPerThread; ++s) {
        const int e = threadIdx.x + s * kThreads;
        if (e < npairs) xstore(g.part + ((size_t)blk * kMaxPairs + e) * 2, tag_part, acc[s]);
    }
    // 2. reduce a share of the entries over all partials, one wave per entry
    if (threadIdx.x == 0) sh.timeout = 0;
    __syncthreads();
    for (int e = (int)blk + (int)nblk * wave; e < npairs; e += (int)nblk * 4) {
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

// R^-1 of the upper-triangular R held in sh.M[0..l-1][0..l-1] into sh.Ri
// (zero below the diagonal), by one wavefront, in 16 x 16 blocks
// R = [R11 R12; 0 R22]: lanes 0..15 back-substitute the columns of R11^-1 and
// lanes 16..31 those of R22^-1 in the same instructions (within a block,
// x_i = -(sum_{t > i} R_it x_t) / R_ii below the diagonal entry
// x_c = 1 / R_cc; rows of the block are broadcast reads from LDS, x is held
// in registers), then the corner -R11^-1 (R12 R22^-1) comes from two 16 x 16
// products on the FP64 matrix cores, the first staged through sh.tile.
// Rows and columns past l act as the identity.
__device__ void inverse_upper(Shared& sh, int l) {
    const int lane = threadIdx.x;   // wave 0, all lanes (the products need the full wave)
    if (lane < 32) sh.dinv[lane] = lane < l ? 1.0 / sh.M[lane][lane] : 1.0;
    __builtin_amdgcn_wave_barrier();
    if (lane < 32) {
        const int o = lane & 16, cc = lane & 15;   // block offset, column within it
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] = 0.0;
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            double s = 0.0;
#pragma unroll
            for (int t = i + 1; t < 16; ++t) {
                const double r = sh.M[o + i][o + t];
                s = fma(o + t < l ? r : 0.0, x[t], s);
            }
            const double di = sh.dinv[o + i];
            x[i] = (i == cc) ? di : (i < cc ? -s * di : 0.0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) sh.Ri[o + i][o + cc] = x[i];
        if (o == 0) {
#pragma unroll
            for (int i = 0; i < 16; ++i) sh.Ri[16 + i][cc] = 0.0;   // below R11^-1
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (l > 16) {   // uniform
        const int li = lane & 15, lk = lane >> 4;
        // P = R12 R22^-1, K = 16 in steps of 4
        v4d pp = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = 4 * s + lk;
            const double a = 16 + k < l ? sh.M[li][16 + k] : 0.0;
            const double b = sh.Ri[16 + k][16 + li];
            pp = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, pp, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) sh.tile[4 * i + lk][li] = pp[i];
        __builtin_amdgcn_wave_barrier();
        // corner = -R11^-1 P
        v4d xc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = 4 * s + lk;
            xc = __builtin_amdgcn_mfma_f64_16x16x4f64(sh.Ri[li][k], sh.tile[k][li], xc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) sh.Ri[4 * i + lk][16 + li] = -xc[i];
    }
    __builtin_amdgcn_wave_barrier();
}

__device__ void cholesky_regs(const OrthArgs& g, Shared& sh, bool detect) {
    const int lane = threadIdx.x;   // wave 0 only
    const int l = g.l;
    if (lane < 32) sh.sel[lane] = 0;
    double Mr[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) Mr[b] = (lane < l && b < l) ? sh.M[lane][b] : 0.0;
    const double myref = lane < l ? sh.M[lane][lane] : 0.0;
    if (lane < l) sh.ref[lane] = myref;
    if (__any(lane < l && !isfinite(myref)) && lane == 0) raise_status(g.ctl, CNMF_ST_NONFINITE);
    const double thr = g.tau2 * wave_max(myref);
    __builtin_amdgcn_wave_barrier();
    bool stop = false;
    double minrat = 1.0;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        if (j < l && !stop) {
            double d = lane_d(Mr[j], j);                     // M[j][j]
            const double wjj = sh.ref[j];
            minrat = fmin(minrat, wjj > 0.0 ? d / wjj : 0.0);
            if (detect) {
                if (!(d > thr)) stop = true;                 // uniform
            } else if (!(d > g.tau2 * sh.ref[j])) {
                if (lane == 0) raise_status(g.ctl, CNMF_ST_BREAKDOWN);
                d = 1.0;
                if (lane > j) Mr[j] = 0.0;
            }
            if (!stop) {
                const double rjj = sqrt(d);
                const double ri = (lane > j && lane < l) ? Mr[j] / rjj : (lane == j ? rjj : 0.0);
                if (lane < 32) {
                    sh.rvec[lane] = ri;
                    sh.M[j][lane] = ri;                      // row j of R
                }
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int b = j + 1; b < 32; ++b) Mr[b] = fma(-ri, sh.rvec[b], Mr[b]);
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    if (lane == 0) sh.minrat = minrat;
    if (stop) {
        if (lane == 0) sh.flag = 1;
        __builtin_amdgcn_wave_barrier();
        return;
    }
    inverse_upper(sh, l);
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
        if (flag == 1 && w == l) {
            // no pool columns in this Gram: report, the caller redoes the
            // factorisation on the augmented Gram
            if (lane == 0) sh.flag = 1;
            __builtin_amdgcn_wave_barrier();
            return;
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
    inverse_upper(sh, l);
}

// Q[r][:] = Ysrc^[r][:] * Ri over this workgroup's rows (FP64 arithmetic):
// tiles of 32 rows staged in LDS (the next tile's loads in flight while the
// current one is multiplied).  Wave (mt, nt) forms the 16 x 16 block of rows
// 16 mt.., columns 16 nt.. of tile * Ri on the FP64 matrix cores, K in steps
// of 4 (Ri is zero below its diagonal; entries past row or column l are
// masked), and, for QT, the transposed block Ri^T tile^T from the same
// operands, whose lanes then hold 16 consecutive rows of one QT column.
__device__ void apply_rows(const OrthArgs& g, Shared& sh, const float* Ysrc, bool use_pool,
                           int64_t r0, int64_t r1, float* Qdst, float* QT) {
    const int l = g.l;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int mt = wave & 1, nt = wave >> 1;
    const int c = 16 * nt + li;          // B operand and Q output column
    const bool active = 16 * nt < l;     // wave-uniform
    constexpr int kPer = (kTile * 32 + kThreads - 1) / kThreads;   // kTile * l <= 4 * kThreads
    float vn[kPer];
    int er[kPer], ec[kPer];
    tile_coords(l, er, ec);
    auto load_tile = [&](int64_t t0) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int rr = er[q], i = ec[q];
            const int64_t r = t0 + rr;
            float v = 0.f;
            if (rr < kTile && r < r1)
                v = (use_pool && sh.sel[i]) ? g.P[r * g.p_rs + i * g.p_cs] : Ysrc[r * l + i];
            vn[q] = v;
        }
    };
    if (r0 < r1) load_tile(r0);
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        lds_barrier();   // every wave is done with the previous tile
#pragma unroll
        for (int q = 0; q < kPer; ++q)
            if (er[q] < kTile) sh.tile[er[q]][ec[q]] = (double)vn[q];
        if (t0 + kTile < r1) load_tile(t0 + kTile);
        lds_barrier();   // LDS only: the loads above and the last stores stay in flight
        if (!active) continue;
        v4d d = {0.0, 0.0, 0.0, 0.0}, dt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int k = 4 * s + lk;
            const double a = k < l ? sh.tile[16 * mt + li][k] : 0.0;
            const double b = (k < l && c < l) ? sh.Ri[k][c] : 0.0;
            d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
            if (QT) dt = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, dt, 0, 0, 0);
        }
        // d: register i holds row 16 mt + 4 i + lk, column c;
        // dt: register i holds column 16 nt + 4 i + lk, row 16 mt + li
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = t0 + 16 * mt + 4 * i + lk;
            if (r < r1 && c < l) Qdst[r * l + c] = (float)d[i];
        }
        if (QT) {
            const int64_t r = t0 + 16 * mt + li;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int col = 16 * nt + 4 * i + lk;
                if (r < r1 && col < l) QT[(int64_t)col * g.ldqt + r] = (float)dt[i];
            }
        }
    }
}

__device__ __forceinline__ void orth_body(const OrthArgs& g, const unsigned blk,
                                          const unsigned nblk) {
    __shared__ Shared sh;
    __syncthreads();   // LDS of a previous panel on this workgroup
    const int64_t rpw = (g.N + nblk - 1) / nblk;
    const int64_t r0 = (int64_t)blk * rpw;
    const int64_t r1 = min(g.N, r0 + rpw);
    const int l = g.l;
    double acc[kPairsPerThread];
    int pa[kPairsPerThread], pb[kPairsPerThread];

    // Stage 0: Gram of Y, Cholesky with the rank test (pass 1).
    // Stage 1 (only if a column of Y is deficient; every workgroup factors
    //   the same sums, so the decision is uniform): the same on the Gram of
    //   [Y P], with the swaps.  Stage 0 or 1 ends with Q1 = Y^ R^-1 in Q.
    // Stage 2 (after stage 1, or when stage 0 found the panel ill-conditioned;
    //   again uniform): Gram of Q1, Cholesky, Q = Q1 R2^-1 in place (pass 2).
    // One loop body keeps a single copy of each step's code.
    if (threadIdx.x == 0) sh.flag = 0;
    int stage = 0;
    while (stage < 3) {
        const bool aug = stage == 1;
        const int w = aug ? 2 * l : l;
        const float* A = stage == 2 ? g.Q : g.Y;
        const unsigned tag = (g.seq << 10) | (unsigned)(2 * stage + 1);
        gram_partial(g, sh, A, w, r0, r1, acc, pa, pb);
        if (!gram_exchange(g, sh, w, tag, tag + 1, acc, pa, pb, blk, nblk)) return;
        if (threadIdx.x < 64) {
            if (aug) cholesky_wave(g, sh, w, true);
            else cholesky_regs(g, sh, stage == 0);
        }
        __syncthreads();
        if (stage == 0 && sh.flag) {
            stage = 1;
            continue;
        }
        if (stage < 2 && blk == 0 && g.replaced && threadIdx.x < l)
            g.replaced[threadIdx.x] = sh.sel[threadIdx.x];
        const bool last = stage == 2 || (stage == 0 && sh.minrat >= kPolish);
        apply_rows(g, sh, A, stage < 2, r0, r1, g.Q, last ? g.QT : nullptr);
        __syncthreads();
        stage = last ? 3 : 2;
    }
}

__global__ __launch_bounds__(kThreads) void k_orth(OrthArgs g) {
    orth_body(g, blockIdx.x, gridDim.x);
}

// Two panels: workgroups [0, a.nblk) factor a, the rest b.
__global__ __launch_bounds__(kThreads) void k_orth2(OrthArgs a, OrthArgs b) {
    if (blockIdx.x < a.nblk) orth_body(a, blockIdx.x, a.nblk);
    else orth_body(b, blockIdx.x - a.nblk, b.nblk);
}

// Batched: workgroup s walks the rounds of sched (instance << 12 | block or
// 0xffffffff); all blocks of a panel share a round and every workgroup is
// resident (the same argument as for the batched subproblem kernel).
__global__ __launch_bounds__(kThreads) void k_orth_batched(const OrthArgs* __restrict__ args,
                                                          const uint32_t* __restrict__ sched,
                                                          int rounds) {
    for (int r = 0; r < rounds; ++r) {
        const uint32_t e = sched[(size_t)r * gridDim.x + blockIdx.x];
        if (e == 0xffffffffu) continue;
        const OrthArgs& g = args[e >> 12];
        orth_body(g, e & 0xfffu, g.nblk);
    }
}

unsigned orth_blocks(const Dev& d, int64_t N) {
    int64_t b = (N + 31) / 32;     // at least 32 rows per workgroup
    if (b > d.num_cus) b = d.num_cus;
    if (b > 256) b = 256;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

size_t orth_exchange_words() { return (size_t)2 * 257 * kMaxPairs * 2; }

size_t orth_batch_exchange_words(unsigned nblk) { return (size_t)(nblk + 1) * kMaxPairs * 2; }

unsigned orth_batch_blocks(int64_t N) {
    const int64_t b = (N + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 256 ? 256 : b));
}

OrthArgs orth_args(int64_t N, int l, const float* Y, const float* pool, bool pool_trans,
                   double tau2, float* Q, float* QT, int64_t ldqt, int32_t* replaced,
                   uint64_t* xch, unsigned seq, Control* ctl, unsigned nblk) {
    OrthArgs g{};
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
    g.nblk = nblk;
    return g;
}

hipError_t orth_batched(const Dev& d, const OrthArgs* args, const uint32_t* sched, int rounds,
                        int slots) {
    if (rounds < 1 || slots < 1) return hipSuccess;
    hipLaunchKernelGGL(k_orth_batched, dim3((unsigned)slots), dim3(kThreads), 0, d.stream, args,
                       sched, rounds);
    return hipGetLastError();
}

unsigned orth_pair_blocks(const Dev& d, int64_t N) {
    const unsigned half = (unsigned)std::max(1, d.num_cus / 2);
    return std::min(orth_blocks(d, N), half);
}

hipError_t orth_pair(const Dev& d, OrthArgs a, OrthArgs b) {
    if (a.N <= 0 || a.l <= 0 || b.N <= 0 || b.l <= 0) return hipErrorInvalidValue;
    if (a.l > 32 || b.l > 32 || a.seq >= (1u << 22) || b.seq >= (1u << 22)) return hipErrorInvalidValue;
    // every workgroup resident (one per compute unit at most): the panels'
    // exchanges wait only on workgroups that are running
    if (a.nblk < 1 || b.nblk < 1 || a.nblk > 256 || b.nblk > 256 ||
        (int)(a.nblk + b.nblk) > d.num_cus)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_orth2, dim3(a.nblk + b.nblk), dim3(kThreads), 0, d.stream, a, b);
    return hipGetLastError();
}

hipError_t orth(const Dev& d, int64_t N, int l, const float* Y, const float* pool,
                bool pool_trans, double tau2, float* Q, float* QT, int64_t ldqt,
                int32_t* replaced, uint64_t* xch, unsigned seq, Control* ctl) {
    if (N <= 0 || l <= 0) return hipSuccess;
    if (l > 32 || seq >= (1u << 22)) return hipErrorInvalidValue;
    const unsigned nb = orth_blocks(d, N);
    const OrthArgs g = orth_args(N, l, Y, pool, pool_trans, tau2, Q, QT, ldqt, replaced, xch, seq,
                                 ctl, nb);
    hipLaunchKernelGGL(k_orth, dim3(nb), dim3(kThreads), 0, d.stream, g);
    return hipGetLastError();
}

}  // namespace cnmf
