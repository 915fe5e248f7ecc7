// One half of a NeNMF outer iteration as one persistent kernel ("phase").
//
// A phase updates one factor by one Nesterov inner loop (Sec. 2): the G
// update of Eq. (2) or the F update of Eq. (3), plain or compressed
// (Sec. 3, Algorithm 1).  In row form both are
//     min_{Z >= 0}  0.5 tr(Z W Z^T) - tr(B^T Z),   grad(Z) = Z W - B,
// over independent rows of p unknowns: the rows of G, or the columns of F.
//
// Inside one launch:
//   1. Small product.  S = sum of the partial products the previous phase
//      left behind (compressed: S = L G or (F R)^T, l x p; plain: S = W).
//      Workgroups split the partial sums, publish their share through
//      tagged slots, and read everyone else's share back.
//   2. W = S^T S (compressed) and L = lambda_max(W) in FP64, computed by
//      every workgroup; B rows = D S with D = X R (G update) or (L X)^T
//      (F update) on the matrix cores (plain: B from an X sweep).
//   3. The inner loop.  Z_k = max(0, Y_k - grad(Y_k)/L), Y_{k+1} = Z_k +
//      ((alpha_{k-1} - 1)/alpha_k)(Z_k - Z_{k-1}), stop at the first k >=
//      inner_min with ||P grad(Z_k)||_F <= tol.  grad(Z_k) = Z_k W - B on the
//      matrix cores, grad(Y) by linearity.  The squared projected-gradient
//      norm of step k is summed in FP64 and published by every workgroup;
//      the test of step k is taken DLAG steps later, so the exchange latency
//      hides behind DLAG further steps whose results are simply discarded
//      when step k turns out to be the last.
//   4. The next phase's partial product over this workgroup's rows:
//      compressed sum_r q_r (x) z_r with q_r the row of Q_L (G update) or
//      Q_R (F update), giving L G = Q_L^T G or (F Q_R)^T; plain Z^T Z.
//
// Layout.  A wave owns TILES tiles of 16 rows.  Lane l holds, for row
// 16 t + (l % 16) of its tiles, the columns c = 16 h + 4 s + l / 16,
// h < PT, s < 4, in register (h, s).  With v_mfma_f32_16x16x4f32 computing
// D' = A Z^T where A[m][k] = W[k][16 h' + perm(m)], perm(m) = 4 (m % 4) +
// m / 4, the B operand of K slice (h, s) is exactly register (h, s), and the
// output register (h', i) lands on column 16 h' + 4 i + l / 16: the product
// Z W comes out in the layout it went in, with no data movement.
//
// Exchange.  Slots are 64-bit words written and read with relaxed
// device-scope atomics: the upper 32 bits carry a tag (launch sequence and
// step), the lower 32 bits the payload, so a reader accepts a word only when
// its tag matches and needs no fence.  An FP64 value takes two words.
#include "internal.hpp"

#include <type_traits>
#include <utility>

namespace cnmf {

namespace {

constexpr int kThreads = 256;
static_assert(kPgSlots >= 2 * 4 + 2, "slots for the largest lag");

__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Moves an MFMA result into vector registers at this point of the program,
// in the MFMA's own basic block, where the compiler spaces the reads from the
// MFMA as the matrix core requires.  A read of the accumulator registers
// placed right after a branch was seen to return a stale element.
__device__ __forceinline__ void settle(v4f& acc) { asm volatile("" : "+v"(acc)); }

__device__ __forceinline__ int perm16(int m) { return 4 * (m & 3) + (m >> 2); }

// Sum over the four lanes that hold one row (l, l ^ 16, l ^ 32, l ^ 48): the
// row swap pairs 16-lane rows 0-1 and 2-3, the half swap the two halves;
// both lanes of a pair add the same two values, so all four hold the same
// bits.
__device__ __forceinline__ float row_sum4(float v) {
    const unsigned b = __float_as_uint(v);
    const auto x = __builtin_amdgcn_permlane16_swap(b, b, false, false);
    const float s = __uint_as_float(x[0]) + __uint_as_float(x[1]);
    const unsigned c = __float_as_uint(s);
    const auto y = __builtin_amdgcn_permlane32_swap(c, c, false, false);
    return __uint_as_float(y[0]) + __uint_as_float(y[1]);
}

__device__ __forceinline__ void slot_store(uint64_t* p, unsigned tag, uint32_t payload) {
    __hip_atomic_store(p, ((uint64_t)tag << 32) | payload, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t slot_load(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// ---------------------------------------------------------------------------
// lambda_max of a symmetric p x p matrix held in LDS as doubles (destroyed),
// by one wavefront: Householder tridiagonalisation (lane i owns row i), then
// Sturm-sequence multisection over 64 points per round.  Returns the value
// on every lane.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lambda_max_wave(double (*A)[33], int p, double* v, double* wv, double* dg,
                                  double* eo) {
    const int lane = threadIdx.x & 63;
    for (int k = 0; k + 2 < p; ++k) {
        const int i = lane;
        const bool in = (i > k) && (i < p);
        const double xi = in ? A[i][k] : 0.0;
        const double sigma = wave_sum(xi * xi);
        const double x0 = A[k + 1][k];
        const double akk = A[k][k];
        if (sigma == 0.0) {
            if (lane == 0) { dg[k] = akk; eo[k] = 0.0; }
            continue;
        }
        const double alpha = -copysign(sqrt(sigma), x0);
        const double v0 = x0 - alpha;
        const double inv = 1.0 / sqrt(sigma - x0 * x0 + v0 * v0);
        const double vi = in ? ((i == k + 1) ? v0 : xi) * inv : 0.0;
        if (in) v[i] = vi;
        __builtin_amdgcn_wave_barrier();
        double ui = 0.0;
        if (in)
            for (int j = k + 1; j < p; ++j) ui = fma(A[i][j], v[j], ui);
        const double c = wave_sum(vi * ui);
        const double wi = 2.0 * (ui - c * vi);
        if (in) wv[i] = wi;
        __builtin_amdgcn_wave_barrier();
        if (in)
            for (int j = k + 1; j < p; ++j) A[i][j] -= vi * wv[j] + wi * v[j];
        if (lane == 0) { dg[k] = akk; eo[k] = alpha; }
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) {
        if (p >= 2) {
            dg[p - 2] = A[p - 2][p - 2];
            eo[p - 2] = A[p - 1][p - 2];
        }
        dg[p - 1] = A[p - 1][p - 1];
    }
    __builtin_amdgcn_wave_barrier();
    // Bracket [lo, hi] around lambda_max: the largest diagonal entry and the
    // Gershgorin bound.  Lane i < p holds row i of the tridiagonal matrix.
    const double di = lane < p ? dg[lane] : -INFINITY;
    const double el = (lane > 0 && lane < p) ? fabs(eo[lane - 1]) : 0.0;
    const double er = (lane + 1 < p) ? fabs(eo[lane]) : 0.0;
    const double lo = wave_max(di);
    const double hi = wave_max(lane < p ? di + el + er : -INFINITY);
    const int bad = __any(lane < p && (!isfinite(di) || !isfinite(er)));
    if (bad) return NAN;
    if (!(hi > 0.0)) return fmax(lo, 0.0);
    // Scale to [.., 1] so the pivots stay O(1), then multisection: 64 Sturm
    // counts per round narrow the bracket 65-fold.
    const double sc = 1.0 / hi;
    double l0 = lo * sc, h0 = 1.0;
    const double pivmin = 1e-300;
    for (int round = 0; round < 9 && h0 > l0; ++round) {
        const double x = l0 + (h0 - l0) * (double)(lane + 1) * (1.0 / 65.0);
        int cnt = 0;   // eigenvalues of T/hi below x (negative LDL^T pivots)
        double q = dg[0] * sc - x;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
        for (int i = 1; i < p; ++i) {
            const double e = eo[i - 1] * sc;
            double r = __builtin_amdgcn_rcp(q);     // 1/q to full precision:
            r = fma(r, fma(-q, r, 1.0), r);         // two Newton steps on the
            r = fma(r, fma(-q, r, 1.0), r);         // hardware estimate
            q = (dg[i] * sc - x) - e * e * r;
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += q < 0.0;
        }
        const unsigned long long mask = __ballot(cnt == p);   // lambda_max < x
        double nlo = l0, nhi = h0;
        if (mask) {
            const int first = __ffsll((long long)mask) - 1;
            nhi = lane_d(x, first);
            if (first > 0) nlo = lane_d(x, first - 1);
        } else {
            nlo = lane_d(x, 63);
        }
        if (!(nhi - nlo < h0 - l0)) break;
        l0 = nlo;
        h0 = nhi;
        if (h0 - l0 <= 1e-13 * h0) break;
    }
    return h0 * hi;
}

}  // namespace

// The warm-started lambda_max below works on one wavefront with lane i < p
// owning row i of the symmetric part of W in FP64 registers (wr) and entry i
// of vectors; everything else is lane reads or row broadcasts (no LDS round
// trips).

// wr = row `lane` of the symmetric W (FP64, LDS, 16-byte aligned rows);
// zero outside p x p.
template <int P>
__device__ __forceinline__ void sym_row(const double (*W)[34], int p, double (&wr)[P]) {
    const int lane = threadIdx.x & 63;
    const int i = lane < P ? lane : 0;
#pragma unroll
    for (int j = 0; j < P; ++j) wr[j] = (lane < p && j < p) ? W[i][j] : 0.0;
}

// v^T W v / v^T v on every lane (lane i < p holds v_i; zero elsewhere).
template <int P>
__device__ __forceinline__ double rayleigh(const double (&wr)[P], double v) {
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int j = 0; j < P; j += 2) {
        t0 = fma(wr[j], lane_d(v, j), t0);
        if (j + 1 < P) t1 = fma(wr[j + 1], lane_d(v, j + 1), t1);
    }
    const double num = wave_sum(v * (t0 + t1));
    const double den = wave_sum(v * v);
    return num / den;
}

// Rayleigh quotient rho = v^T W v / v^T v and the squared residual
// ||W v - rho v||^2 / v^T v, on every lane.
template <int P>
__device__ __forceinline__ double rayleigh_res(const double (&wr)[P], double v, double& res2) {
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int j = 0; j < P; j += 2) {
        t0 = fma(wr[j], lane_d(v, j), t0);
        if (j + 1 < P) t1 = fma(wr[j + 1], lane_d(v, j + 1), t1);
    }
    const double wv = t0 + t1;                 // (W v)_lane; 0 on lanes >= p
    const double den = wave_sum(v * v);
    const double rho = wave_sum(v * wv) / den;
    const double r = fma(-rho, v, wv);
    res2 = wave_sum(r * r) / den;
    return rho;
}

// v scaled to (about) unit length: only its direction is used
__device__ __forceinline__ void normalise(double& v) {
    const double nn = wave_sum(v * v);
    v *= (nn > 0.0 && nn < 1e300) ? __builtin_amdgcn_rsq(nn) : 0.0;
}

// Lane k's value of v on every lane of its 16-lane row (DPP row_newbcast).
template <int K>
__device__ __forceinline__ float row_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + K, 0xf, 0xf, true));
}
template <class F, int... K>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, K...>) {
    (f(std::integral_constant<int, K>{}), ...);
}
// f(integral_constant<int, k>) for k = 0 .. N - 1, in order
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// shifted_solve (below) for p <= 16: the rows live in lanes 0..15, one DPP
// row, so the pivot row travels by row broadcasts instead of lane reads into
// scalar registers; the counts are taken from lane 0, whose row holds the
// system (lanes 16..63 run the same steps on zero rows).
__device__ __forceinline__ int shifted_solve16(const double (&wr)[16], double sigma, double& x, int p) {
    const int lane = threadIdx.x & 63;
    float R[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) R[c] = lane < p ? (float)(wr[c] - (lane == c ? sigma : 0.0)) : 0.f;
    float ri = lane < p ? (float)x : 0.f;
    float inv_own = 0.f;
    int neg = 0;
    bool bad = false;
    static_for<16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const bool kin = k < p;
        const float d = row_bcast<k>(R[k]);
        neg += kin && d < 0.f;
        const bool good = d != 0.f && fabsf(d) < 1e37f;
        bad = bad || (kin && !good);
        const float inv = __builtin_amdgcn_rcpf(good ? d : 1.f);
        if (lane == k) inv_own = kin ? inv : 0.f;
        const float f = (kin && lane > k) ? R[k] * inv : 0.f;
        ri = fmaf(-f, row_bcast<k>(ri), ri);
#pragma unroll
        for (int c = k + 1; c < 16; ++c) R[c] = fmaf(-f, row_bcast<k>(R[c]), R[c]);
    });
    float xi = 0.f;
    float acc = ri;
    static_for<16>([&](auto kc) {
        constexpr int k = 15 - decltype(kc)::value;
        const float xk = row_bcast<k>(acc * inv_own);
        if (lane == k) xi = xk;
        if (lane < k) acc = fmaf(-R[k], xk, acc);
    });
    x = lane < p ? (double)xi : 0.0;
    neg = __builtin_amdgcn_readfirstlane(neg);
    bad = __builtin_amdgcn_readfirstlane((int)bad) != 0;
    return bad ? -1 : neg;
}

// Solves (W - sigma I) x = r by Gaussian elimination without pivoting in
// FP32, fully unrolled over the P columns: lane i keeps row i in registers
// (R[c] = M[i][c]); at step k the pivot row is read from lane k and every
// lane below subtracts its multiple.  A lane's row no longer changes once it
// has been the pivot, so at the end lane i holds row i of the upper factor,
// which the back substitution reads in place.  Returns the number of
// negative pivots -- by Sylvester's law of inertia the number of
// eigenvalues of W below sigma -- or -1 on a zero or non-finite pivot.
// x: right-hand side in, solution out (lane-distributed).  FP32 suffices for
// the count whenever sigma is separated from the spectrum by much more than
// p eps32 ||W|| (the elimination of a definite matrix is backward stable);
// x only needs to be a good direction, so the pivots are inverted with the
// hardware reciprocal.
template <int P>
__device__ __forceinline__ int shifted_solve(const double (&wr)[P], double sigma, double& x, int p) {
    if constexpr (P == 16) {
        return shifted_solve16(wr, sigma, x, p);
    } else {
        const int lane = threadIdx.x & 63;
        float R[P];
#pragma unroll
        for (int c = 0; c < P; ++c) R[c] = lane < p ? (float)(wr[c] - (lane == c ? sigma : 0.0)) : 0.f;
        float ri = lane < p ? (float)x : 0.f;
        float inv_own = 0.f;   // lane k: 1 / pivot k
        int neg = 0;
        bool bad = false;
        // static trip counts (full unroll, no register indexing); steps k >= p
        // change nothing
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const bool kin = k < p;
            const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(R[k]), k));
            neg += kin && d < 0.f;
            const bool good = d != 0.f && fabsf(d) < 1e37f;
            bad = bad || (kin && !good);
            const float inv = __builtin_amdgcn_rcpf(good ? d : 1.f);
            if (lane == k) inv_own = kin ? inv : 0.f;
            const float f = (kin && lane > k) ? R[k] * inv : 0.f;
            ri = fmaf(-f, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ri), k)), ri);
#pragma unroll
            for (int c = k + 1; c < P; ++c)
                R[c] = fmaf(-f, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(R[c]), k)), R[c]);
        }
        // back substitution: once x_k is known, every lane i < k removes U[i][k] x_k
        float xi = 0.f;
        float acc = ri;
#pragma unroll
        for (int k = P - 1; k >= 0; --k) {   // lanes k >= p hold acc = inv_own = 0
            const float xk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc * inv_own), k));
            if (lane == k) xi = xk;
            if (lane < k) acc = fmaf(-R[k], xk, acc);
        }
        x = lane < p ? (double)xi : 0.0;
        return bad ? -1 : neg;
    }
}

// lambda_max of the symmetric W (p x p, FP64 in LDS) by one wavefront,
// warm-started from the top eigenvector of the previous subproblem of the
// same side (prev_L <= 0 means none; lane i < p holds its component i in
// prev_v).  One inverse-iteration step from that vector, with the shift
// sigma = rho0 (1 + 1e-4) just above its Rayleigh quotient rho0 (FP32
// elimination of W - sigma I), gives v; rho = Rayleigh(v) <= lambda_max.
// The Kato-Temple inequality bounds the rest: if every other eigenvalue is
// at most a < rho, then lambda_max <= rho + ||W v - rho v||^2 / (rho - a).
// W is symmetric positive semidefinite up to the rounding of its entries,
// so lambda_2 <= trace(W) - lambda_max + (rounding) <= trace(W) - rho + 1e-4
// trace(W) = a.  When that bound is within 1e-12 rho of rho, L = the bound:
// an upper bound of lambda_max within 1e-12 relative.  Otherwise (no start,
// no separation of lambda_max from the rest, a vector not yet accurate
// enough) the tridiagonalisation and bisection above (on M, LDS) give L, the
// upper end of a bracket 1e-13 wide, and one inverse-iteration step gives
// the vector.  On return v (lane-distributed) is the unit top eigenvector.
template <int P>
__device__ __forceinline__ double lambda_max_warm(const double (*W)[34], double (*M)[33], int p,
                                                  double prev_L, double prev_v, double& v,
                                                  double* wv, double* dg, double* eo, double* tv) {
    const int lane = threadIdx.x & 63;
    double wr[P];
    sym_row<P>(W, p, wr);
    if (prev_L > 0.0) {
        v = lane < p ? prev_v : 0.0;
        const double rho0 = rayleigh<P>(wr, v);
        if (rho0 > 0.0 && rho0 < 1e300) {
            const int cnt = shifted_solve<P>(wr, rho0 * (1.0 + 1e-4), v, p);
            normalise(v);
            double res2 = 0.0;
            const double rho = rayleigh_res<P>(wr, v, res2);
            const double tr = wave_sum(lane < p ? W[lane][lane] : 0.0);
            const double gap = rho - (tr - rho) - 1e-4 * fabs(tr);   // rho - a
            if (cnt >= 0 && gap > 0.0 && rho < 1e300 && res2 <= 1e-12 * rho * gap)
                return rho + res2 / gap;
        }
    }
    if (lane < p)
#pragma unroll
        for (int j = 0; j < P; ++j) M[lane][j] = wr[j];
    __builtin_amdgcn_wave_barrier();
    const double L = lambda_max_wave(M, p, tv, wv, dg, eo);
    v = lane < p ? 1.0 : 0.0;
    if (L > 0.0 && L < 1e300) {
        shifted_solve<P>(wr, L * (1.0 + 1e-5), v, p);
        normalise(v);
    } else {
        v = 0.0;
    }
    return L;
}

namespace {

// What a workgroup carries from one phase of a side to the next inside the
// fused outer loop: the warm start of lambda_max (wave 0: L, and component
// `lane` of the eigenvector) and the running bound of the global rule.
struct PhaseState {
    double eig_L, eig_v, tol;
};

// One subproblem (G rows or F columns) on workgroup blk of nblk; seq tags
// the exchange words of this launch.  st (fused outer loop only) replaces the
// warm start read from eig_in / written to eig_out and the running bound
// read from tol_ptr / written to tol_state.
// SOLVER: kSolverNesterov (Sec. 2), kSolverRestart (the same loop with the
// momentum of every row restarted adaptively; non-grouped exchange only),
// kSolverHals or kSolverMu (fixed counts of HALS sweeps or multiplicative
// updates; no Lipschitz constant, no stopping test).
template <int PT, int TILES, int DLAG, int SOLVER = kSolverNesterov>
__device__ __forceinline__ void phase_body(const PhaseArgs& a, const unsigned blk,
                                           const unsigned nblk, const unsigned seq,
                                           PhaseState* st = nullptr) {
    constexpr bool ALT = SOLVER == kSolverHals || SOLVER == kSolverMu;
    constexpr bool RESTART = SOLVER == kSolverRestart;
    static_assert(!RESTART || DLAG != kGrouped, "restart runs the per-step exchange");
    // DLAG = kGrouped: the norms of GB consecutive steps travel in one
    // exchange, tested one group late; otherwise every step's norm is
    // exchanged and tested DLAG steps late.
    constexpr bool GROUPED = DLAG == kGrouped;
    constexpr int GB = 4;
    constexpr int NH = GROUPED ? 2 : ((DLAG + 1) > 2 ? (DLAG + 1) : 2);   // iterates kept
    constexpr int NR = PT * 4;                              // registers per row tile
    // exchanges in flight (grouped: a workgroup that publishes group h has
    // tested group h - 1, so every workgroup has read group h - 2)
    constexpr int NSLOT = GROUPED ? 4 : 2 * DLAG + 2;
    static_assert((size_t)NSLOT * 256 * 2 * (GROUPED ? GB : 1) <= kPgWords, "exchange words");
    __shared__ float sS[32][33];      // S (rows: M index, cols: p)
    __shared__ float sW[32][33];      // W (p x p)
    __shared__ __align__(16) double sWd[32][34];   // (W + W^T) / 2 in FP64, for lambda_max
    __shared__ double sv[32], swv[32], sdg[32], seo[32];
    __shared__ double sM[32][33];     // work matrix of the eigenvalue solver
    __shared__ double s_red[4];
    __shared__ double s_pub[2][4][GB];    // grouped, by group parity: wave sums of own norms
    __shared__ double s_cons[2][4][GB];   //   wave sums of the polled norms
    __shared__ __align__(16) int s_cok[2][4];   //   polled words all carried the group's tag
    __shared__ double s_tot;
    __shared__ double s_L;
    __shared__ int s_flag;
    __shared__ float zt[4][16][33];   // per-wave transpose tile
    __shared__ float sred[4][16][64]; // epilogue reduction
    __shared__ float sbeta[RESTART ? kBetaLds : 1];   // momentum weights by a row's own step

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int q16 = lane & 15;
    const int g4 = lane >> 4;
    const int p = a.p;
    // a time-budgeted loop whose deadline has passed: nothing left to do (the
    // flag was written by an earlier launch, so every workgroup sees it)
    if (a.stop_flag && *a.stop_flag) return;
    // LDS of a previous subproblem on this workgroup (global stores of the
    // previous phase stay in flight: nothing here reads them back)
    lds_barrier();
    if constexpr (RESTART)
        for (int e = threadIdx.x; e < kBetaLds; e += kThreads) sbeta[e] = a.beta[e];
    Control* ctl = a.ctl;
    bool ok = true;
    // warm start of lambda_max (wave 0), fetched now so the load is in
    // flight during the exchange of S
    double eig_L = 0.0, eig_v = 0.0;
    if (st) {
        if (a.kind == 0 && wave == 0) {
            eig_L = st->eig_L;
            eig_v = lane < p ? st->eig_v : 0.0;
        }
    } else if (a.kind == 0 && a.eig_in && wave == 0) {
        eig_L = a.eig_in[0];
        const double e = a.eig_in[1 + (lane < p ? lane : p - 1)];
        eig_v = lane < p ? e : 0.0;
    }

    // ---------------- 0. row loads ------------------------------------------
    // Z rows, D rows and the Q operand do not depend on S: their loads are
    // issued first, so they are in flight during the exchange of S and
    // lambda_max.
    const int64_t row_base = (int64_t)blk * (64 * TILES) + (int64_t)wave * (16 * TILES);
    float z[TILES][NR], bb[TILES][NR];
    float dv[TILES][2][4];   // D[r][k], k = 16 hk + 4 s + l / 16 (mode 2)
    // Loads are unconditional, from indexes clamped into the operands, and
    // masked afterwards: no divergent branches, so they all issue back to back.
    const int64_t rlast = a.rows > 0 ? a.rows - 1 : 0;
    const bool has_rows = a.rows > 0;
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
        const int64_t r = row_base + 16 * t + q16;
        const bool act = r < a.rows;
        const int64_t rc = act ? r : rlast;
#pragma unroll
        for (int h = 0; h < PT; ++h)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int c = 16 * h + 4 * s + g4;
                const int cc = c < p ? c : p - 1;
                const bool in = act && c < p;
                const float zv = has_rows ? a.Z[rc * a.z_rs + cc * a.z_cs] : 0.f;
                z[t][4 * h + s] = in ? zv : 0.f;
                const float bv = (has_rows && a.mode != 2) ? a.Bgiven[rc * p + cc] : 0.f;
                bb[t][4 * h + s] = in ? bv : 0.f;
            }
#pragma unroll
        for (int hk = 0; hk < 2; ++hk)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 16 * hk + 4 * s + g4;
                const int kc = k < a.ell ? k : a.ell - 1;
                const float d = (has_rows && a.mode == 2) ? a.D[rc * a.d_rs + kc * a.d_cs] : 0.f;
                dv[t][hk][s] = (act && k < a.ell) ? d : 0.f;
            }
    }

    // Q operand of the closing product (mode 2), fetched now so that its
    // latency hides behind the inner loop (small tile counts only: registers)
    constexpr bool QPRE = TILES <= 2;
    float qpre[QPRE ? TILES : 1][4][2];
    if constexpr (QPRE) {
#pragma unroll
        for (int t = 0; t < TILES; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int hm = 0; hm < 2; ++hm) {
                    const int64_t r = row_base + 16 * t + 4 * s + g4;
                    const int k = 16 * hm + q16;
                    const int64_t rc = r < a.rows ? r : rlast;
                    const int kc = k < a.ell ? k : a.ell - 1;
                    const float qv = (has_rows && a.mode == 2 && (a.part_out || a.part_out64)) ? a.Q[rc * a.ell + kc] : 0.f;
                    qpre[t][s][hm] = (r < a.rows && k < a.ell) ? qv : 0.f;
                }
    }

    // ---------------- 1. small product S ------------------------------------
    const int Srows = (a.mode == 2) ? a.ell : p;
    const int nS = Srows * p;
    for (int e = threadIdx.x; e < 32 * 33; e += kThreads) {
        sS[e / 33][e % 33] = 0.f;
        sW[e / 33][e % 33] = 0.f;
    }
    __syncthreads();
    if (a.mode == 0) {
        for (int e = threadIdx.x; e < p * p; e += kThreads) {
            const int i = e / p, j = e % p;
            sW[i][j] = a.Wgiven[e];
            sWd[i][j] = 0.5 * ((double)a.Wgiven[e] + (double)a.Wgiven[j * p + i]);
        }
    } else if (a.kind != 2) {
        // this workgroup's share: entries e = blk + nblk * j, one wave each
        for (int e = (int)blk + (int)nblk * wave; e < nS; e += (int)nblk * 4) {
            const int mr = e / p, nc = e % p;
            double t = 0.0;
            if (a.part_in64) {
                // tagged partials of the phase before, written in this launch
                for (int j = lane; j < a.nin; j += 64) {
                    const uint64_t* wp = &a.part_in64[(size_t)j * 1024 + mr * 32 + nc];
                    uint64_t w = slot_load(wp);
                    unsigned spins = 0;
                    while ((unsigned)(w >> 32) != a.seq_in) {
                        __builtin_amdgcn_s_sleep(1);
                        if ((++spins & 255u) == 0u &&
                            (spins >= kSpinLimit || (atomic_status_load(&ctl->status) & CNMF_ST_TIMEOUT))) {
                            raise_status(ctl, CNMF_ST_TIMEOUT);
                            break;
                        }
                        w = slot_load(wp);
                    }
                    t += (double)__uint_as_float((uint32_t)w);
                }
            } else {
                for (int j = lane; j < a.nin; j += 64) t += (double)a.part_in[(size_t)j * 1024 + mr * 32 + nc];
            }
            t = wave_sum(t);
            if (lane == 0) slot_store(&a.slot_s[e], seq, __float_as_uint((float)t));
        }
        // read all shares back
        unsigned spins = 0;
        for (;;) {
            int mine_ok = 1;
            for (int e = threadIdx.x; e < nS; e += kThreads) {
                const uint64_t w = slot_load(&a.slot_s[e]);
                if ((unsigned)(w >> 32) == seq) sS[e / p][e % p] = __uint_as_float((uint32_t)w);
                else mine_ok = 0;
            }
            if (__syncthreads_and(mine_ok)) break;
            __builtin_amdgcn_s_sleep(1);
            ++spins;
            int to = 0;
            if (threadIdx.x == 0 && (spins & 255u) == 0u)
                to = spins >= (kSpinLimit >> 4) || (atomic_status_load(&ctl->status) & CNMF_ST_TIMEOUT);
            if (__syncthreads_or(to)) {
                if (threadIdx.x == 0) raise_status(ctl, CNMF_ST_TIMEOUT);
                ok = false;
                break;
            }
        }
        if (a.mode == 1) {
            for (int e = threadIdx.x; e < p * p; e += kThreads) {
                const int i = e / p, j = e % p;
                sW[i][j] = sS[i][j];
                sWd[i][j] = 0.5 * ((double)sS[i][j] + (double)sS[j][i]);
            }
        } else {
            // W = S^T S (l x p -> p x p), FP64 accumulation in k order
            // (unrolled so that the LDS reads issue ahead of the chain)
            for (int e = threadIdx.x; e < p * p; e += kThreads) {
                const int i = e / p, j = e % p;
                double t = 0.0;
#pragma unroll 8
                for (int k = 0; k < a.ell; ++k) t = fma((double)sS[k][i], (double)sS[k][j], t);
                sW[i][j] = (float)t;
                // lambda_max is taken of the FP32 W that the gradient uses (its
                // Lipschitz constant), held exactly in FP64; symmetric: (i, j)
                // and (j, i) sum alike
                sWd[i][j] = (double)(float)t;
            }
        }
    }
    __syncthreads();

    // ---------------- 2. B rows, Lipschitz constant (wave 0) ----------------

    // A operand of the gradient product: W[k][16h' + perm(m)] (Z W) or its
    // transpose (Z W^T), k = 16 h + 4 s + l / 16, m = l % 16.
    float wA[PT][PT][4];
#pragma unroll
    for (int hp = 0; hp < PT; ++hp)
#pragma unroll
        for (int h = 0; h < PT; ++h)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 16 * h + 4 * s + g4;
                const int c = 16 * hp + perm16(q16);
                wA[hp][h][s] = a.wt ? sW[c][k] : sW[k][c];
            }

    double L = 1.0;
    if (!ALT && a.kind == 0 && wave == 0) {
        double ev;
        const double lm = lambda_max_warm<16 * PT>(sWd, sM, p, eig_L, eig_v, ev, swv, sdg, seo, sv);
        if (lane == 0) s_L = lm;
        if (st) {
            st->eig_L = (lm > 0.0 && lm == lm) ? lm : 0.0;
            st->eig_v = lane < p ? ev : 0.0;
        } else if (a.eig_out && blk == 0) {
            if (lane == 0) a.eig_out[0] = (lm > 0.0 && lm == lm) ? lm : 0.0;
            if (lane < p) a.eig_out[1 + lane] = ev;
        }
    }
    if (a.kind == 0 && a.w_out && blk == 0 && wave == 1)
        for (int e = lane; e < p * p; e += 64) a.w_out[e] = sW[e / p][e % p];

    if (a.mode == 2) {
        // B rows = D S: A operand S[k][16h' + perm(m)], B operand D[r][k]
#pragma unroll
        for (int t = 0; t < TILES; ++t)
#pragma unroll
            for (int hp = 0; hp < PT; ++hp) {
                v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int hk = 0; hk < 2; ++hk)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int k = 16 * hk + 4 * s + g4;
                        const int c = 16 * hp + perm16(q16);
                        const float av = (k < a.ell && c < p) ? sS[k][c] : 0.f;
                        acc = mfma16(av, dv[t][hk][s], acc);
                    }
                settle(acc);
#pragma unroll
                for (int i = 0; i < 4; ++i) bb[t][4 * hp + i] = acc[i];
            }
    }

    auto grad = [&](const float (&zz)[NR], const float (&b)[NR], float (&g)[NR]) {
#pragma unroll
        for (int hp = 0; hp < PT; ++hp) {
            v4f acc = {-b[4 * hp + 0], -b[4 * hp + 1], -b[4 * hp + 2], -b[4 * hp + 3]};
#pragma unroll
            for (int h = 0; h < PT; ++h)
#pragma unroll
                for (int s = 0; s < 4; ++s) acc = mfma16(wA[hp][h][s], zz[4 * h + s], acc);
            settle(acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) g[4 * hp + i] = acc[i];
        }
    };
    auto pg2_of = [&](const float (&zz)[NR], const float (&g)[NR]) {
        double sacc = 0.0;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const float pg = (zz[i] > 0.f) ? g[i] : fminf(g[i], 0.f);
            const double d = (g[i] != g[i]) ? (double)g[i] : (double)pg;
            sacc = fma(d, d, sacc);
        }
        return sacc;
    };
    // workgroup sum of one double per thread, published as step `step`
    auto publish = [&](double v, int step) {
        v = wave_sum(v);
        if (lane == 0) s_red[wave] = v;
        lds_barrier();
        if (threadIdx.x == 0) {
            const double tot = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
            const uint64_t bits = (uint64_t)__double_as_longlong(tot);
            const unsigned tag = (seq << 10) | ((unsigned)step & 1023u);
            uint64_t* sl = a.slot_pg + ((size_t)(step % NSLOT) * 256 + blk) * 2;
            slot_store(sl + 0, tag, (uint32_t)(bits >> 32));
            slot_store(sl + 1, tag, (uint32_t)(bits & 0xffffffffu));
        }
    };
    // Poll words of step `step`, issued early by wave 0 (up to 256 workgroups,
    // four per lane) and checked later by collect().
    uint64_t pwA[4][2];
    auto poll_issue = [&](int step, uint64_t (&pw)[4][2]) {
        const uint64_t* base = a.slot_pg + (size_t)(step % NSLOT) * 256 * 2;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const unsigned i = lane + 64 * u;
            const unsigned ic = i < nblk ? i : 0u;
            pw[u][0] = slot_load(base + 2 * ic);
            pw[u][1] = slot_load(base + 2 * ic + 1);
        }
    };
    // grid total of step `step` (wave 0 polls; result broadcast through LDS);
    // prefetched: start from the words poll_issue() loaded
    auto collect = [&](int step, bool prefetched, const uint64_t (&pw)[4][2]) -> double {
        if (wave == 0) {
            const unsigned tag = (seq << 10) | ((unsigned)step & 1023u);
            const uint64_t* base = a.slot_pg + (size_t)(step % NSLOT) * 256 * 2;
            unsigned spins = 0;
            int to = 0;
            double t = 0.0;
            bool first = prefetched;
            for (;;) {
                int mine_ok = 1;
                t = 0.0;
                if (first) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const unsigned i = lane + 64 * u;
                        if (i < nblk) {
                            const uint64_t w0 = pw[u][0], w1 = pw[u][1];
                            if ((unsigned)(w0 >> 32) == tag && (unsigned)(w1 >> 32) == tag)
                                t += __longlong_as_double((long long)((w0 << 32) | (w1 & 0xffffffffu)));
                            else
                                mine_ok = 0;
                        }
                    }
                    first = false;
                } else {
                    for (unsigned i = lane; i < nblk; i += 64) {
                        const uint64_t w0 = slot_load(base + 2 * i);
                        const uint64_t w1 = slot_load(base + 2 * i + 1);
                        if ((unsigned)(w0 >> 32) == tag && (unsigned)(w1 >> 32) == tag)
                            t += __longlong_as_double((long long)((w0 << 32) | (w1 & 0xffffffffu)));
                        else
                            mine_ok = 0;
                    }
                }
                if (__all(mine_ok)) break;
                __builtin_amdgcn_s_sleep(1);
                ++spins;
                int t0 = 0;
                if ((spins & 255u) == 0u)
                    t0 = spins >= (kSpinLimit >> 4) ||
                         (atomic_status_load(&ctl->status) & CNMF_ST_TIMEOUT);
                if (__any(t0)) { to = 1; break; }
            }
            t = wave_sum(t);
            if (lane == 0) {
                s_tot = t;
                s_flag = to;
                if (to) raise_status(ctl, CNMF_ST_TIMEOUT);
            }
        }
        lds_barrier();
        return s_tot;
    };

    float g[TILES][NR];
#pragma unroll
    for (int t = 0; t < TILES; ++t) grad(z[t], bb[t], g[t]);

    __syncthreads();   // s_L
    L = (a.kind == 0) ? s_L : 1.0;

    const bool need_pg0 = a.kind != 2 && (a.kind == 1 || a.pg2_out != nullptr || a.ratio > 0.0);
    double pg0 = 0.0;
    if (need_pg0 && ok) {
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < TILES; ++t) v += pg2_of(z[t], g[t]);
        publish(v, 0);
        pg0 = collect(0, false, pwA);
        if (s_flag) ok = false;
    }

    double tol = st ? st->tol : (a.tol_ptr ? *a.tol_ptr : a.tol_value);
    if (a.ratio > 0.0 && a.kind == 0) tol = a.ratio * sqrt(pg0);
    const double tol2 = tol >= 0.0 ? tol * tol : -1.0;   // the test is ||pg||^2 <= tol^2
    const int forced = a.forced_ptr ? (int)*a.forced_ptr : a.forced;
    const int kmax = (a.kind != 0) ? 0 : (forced >= 0 ? forced : a.inner_max);
    int steps = 0;

    // zh[j] = Z_{K - j}
    float zh[NH][TILES][NR];
#pragma unroll
    for (int j = 0; j < NH; ++j)
#pragma unroll
        for (int t = 0; t < TILES; ++t)
#pragma unroll
            for (int i = 0; i < NR; ++i) zh[j][t][i] = z[t][i];
    int out_idx = GROUPED ? -1 : 0;   // the grouped loop writes z itself

    if constexpr (ALT) {
        if (ok && kmax > 0) {
            if constexpr (SOLVER == kSolverHals) {
                // Coordinate j of a row lives in register j / 4 of the lane
                // with g4 = j % 4 (column 4 r + g4 in register r); the row's
                // four lanes add their shares of grad_j and the owner moves
                // z_j to the minimiser along j, clipped at 0 (Gauss-Seidel:
                // the next coordinate sees the new value).
                for (int it = 0; it < kmax; ++it) {
#pragma unroll
                    for (int j = 0; j < 16 * PT; ++j) {
                        if (j >= p) continue;   // uniform
                        const int r = j >> 2;
                        const bool own = g4 == (j & 3);
                        const float wjj = sW[j][j];
                        float ca[NR];
#pragma unroll
                        for (int rr = 0; rr < NR; ++rr)
                            ca[rr] = a.wt ? sW[j][4 * rr + g4] : sW[4 * rr + g4][j];
#pragma unroll
                        for (int t = 0; t < TILES; ++t) {
                            float dsum = 0.f;
#pragma unroll
                            for (int rr = 0; rr < NR; ++rr) dsum = fmaf(z[t][rr], ca[rr], dsum);
                            dsum = row_sum4(dsum);
#pragma unroll
                            for (int rr = 0; rr < NR; ++rr) {
                                if (rr != r) continue;
                                if (own && wjj > 0.f) {
                                    const float nz = z[t][rr] - (dsum - bb[t][rr]) / wjj;
                                    z[t][rr] = (nz > 0.f || nz != nz) ? nz : 0.f;
                                }
                            }
                        }
                    }
                }
            } else {
                // Z <- Z * sqrt((B+ + Z A-) / (B- + Z A+)) with A the operand
                // of the gradient product (W, or W^T for F): both products on
                // the matrix cores in the layout of Z.
                float wAp[PT][PT][4], wAn[PT][PT][4];
#pragma unroll
                for (int hp = 0; hp < PT; ++hp)
#pragma unroll
                    for (int h = 0; h < PT; ++h)
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            wAp[hp][h][s] = fmaxf(wA[hp][h][s], 0.f);
                            wAn[hp][h][s] = fmaxf(-wA[hp][h][s], 0.f);
                        }
                auto prod = [&](const float (&op)[PT][PT][4], const float (&zz)[NR], float (&o)[NR]) {
#pragma unroll
                    for (int hp = 0; hp < PT; ++hp) {
                        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int h = 0; h < PT; ++h)
#pragma unroll
                            for (int s = 0; s < 4; ++s) acc = mfma16(op[hp][h][s], zz[4 * h + s], acc);
                        settle(acc);
#pragma unroll
                        for (int i = 0; i < 4; ++i) o[4 * hp + i] = acc[i];
                    }
                };
                for (int it = 0; it < kmax; ++it) {
#pragma unroll
                    for (int t = 0; t < TILES; ++t) {
                        float zp[NR], zm[NR];
                        prod(wAp, z[t], zp);
                        prod(wAn, z[t], zm);
#pragma unroll
                        for (int i = 0; i < NR; ++i) {
                            const float num = fmaxf(bb[t][i], 0.f) + zm[i];
                            const float den = fmaxf(-bb[t][i], 0.f) + zp[i];
                            const float ratio = den > 0.f ? num / den : 1.f;
                            z[t][i] *= sqrtf(ratio);
                        }
                    }
                }
            }
        }
        steps = kmax;
        out_idx = -1;   // z holds the result
    } else {
    if (!(L > 0.0)) {
        if (a.kind == 0 && blk == 0 && threadIdx.x == 0)
            raise_status(ctl, (L != L) ? CNMF_ST_NONFINITE : CNMF_ST_ZERO_LIPS);
    } else if (ok && kmax > 0) {
        const float invL = (float)(1.0 / L);
        float gp[TILES][NR];
#pragma unroll
        for (int t = 0; t < TILES; ++t)
#pragma unroll
            for (int i = 0; i < NR; ++i) gp[t][i] = g[t][i];
        float beta = 0.f;   // momentum weight of the next step (non-grouped loop)
        const bool check = forced < 0;
        int stop_at = -1;
        int K = 1;
        int kend = kmax;
        if constexpr (GROUPED) {
            // Steps run in groups of GB: group gi holds steps GB (gi-1) + 1 .. GB gi.
            // The norm of step K - 1 is formed while the products of step K run.
            // A group's norms are published together at the first step of the
            // next group; they are polled at the second step and tested at the
            // last step of the GLAG-th group after theirs, so a stop at step s
            // is seen at most (GLAG + 1) GB - 1 steps later; the iterates of the
            // group under test are kept for the return value.
            static_assert(GB == 4, "four norms per exchange");
            constexpr int POLL_AT = 1, TEST_AT = GB - 1;   // steps of the group after the publish
            constexpr int GLAG = 2;                          // groups between a group and its test
            const int glast = (kmax + GB - 1) / GB;
            const int q = quad_slot(lane);            // step of a group this lane reduces
            float cur[GB][TILES][NR], sav[GB][TILES][NR], gb2[2][TILES][NR];
            float sav2[GLAG > 1 ? GB : 1][TILES][NR];   // the group before sav (GLAG = 2)
            double pgv[GB];
            uint64_t pw[4][2];
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                pgv[u] = 0.0;
#pragma unroll
                for (int t = 0; t < TILES; ++t)
#pragma unroll
                    for (int i = 0; i < NR; ++i) sav[u][t][i] = z[t][i];
            }
#pragma unroll
            for (int t = 0; t < TILES; ++t)
#pragma unroll
                for (int i = 0; i < NR; ++i) gb2[0][t][i] = gb2[1][t][i] = g[t][i];
            auto testable = [&](int gc) { return gc >= 1 && gc * GB >= a.inner_min; };
            auto poll_group = [&](int gc) {
                const uint64_t* base = a.slot_pg + (size_t)(gc % NSLOT) * 256 * (2 * GB) + 2 * q;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const unsigned i = (unsigned)(wave * 64 + 16 * j + (lane >> 2));
                    const unsigned ic = i < nblk ? i : 0u;
                    pw[j][0] = slot_load(base + (size_t)ic * (2 * GB));
                    pw[j][1] = slot_load(base + (size_t)ic * (2 * GB) + 1);
                }
            };
            auto publish_group = [&](int gc) {
                const double r = wave_sum4(pgv);
                if (lane < GB) s_pub[gc & 1][wave][q] = r;
                lds_barrier();
                if (threadIdx.x < GB) {
                    const int uu = threadIdx.x;
                    const double tot = (s_pub[gc & 1][0][uu] + s_pub[gc & 1][1][uu]) +
                                       (s_pub[gc & 1][2][uu] + s_pub[gc & 1][3][uu]);
                    const uint64_t bits = (uint64_t)__double_as_longlong(tot);
                    const unsigned tag = (seq << 10) | ((unsigned)gc & 1023u);
                    uint64_t* sl = a.slot_pg + ((size_t)(gc % NSLOT) * 256 + blk) * (2 * GB) + 2 * uu;
                    slot_store(sl, tag, (uint32_t)(bits >> 32));
                    slot_store(sl + 1, tag, (uint32_t)(bits & 0xffffffffu));
                }
            };
            // grid totals of group gc's norms; false on time-out
            auto consume_group = [&](int gc, double (&tot)[GB]) -> bool {
                const unsigned tag = (seq << 10) | ((unsigned)gc & 1023u);
                const int par = gc & 1;
                for (unsigned spins = 0;; ++spins) {
                    int okl = 1;
                    double pj[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const unsigned i = (unsigned)(wave * 64 + 16 * j + (lane >> 2));
                        const uint64_t w0 = pw[j][0], w1 = pw[j][1];
                        const bool good = (unsigned)(w0 >> 32) == tag && (unsigned)(w1 >> 32) == tag;
                        pj[j] = (i < nblk && good)
                                    ? __longlong_as_double((long long)((w0 << 32) | (w1 & 0xffffffffu)))
                                    : 0.0;
                        if (i < nblk && !good) okl = 0;
                    }
                    double r = (pj[0] + pj[1]) + (pj[2] + pj[3]);
                    r += dpp_d<kDppRor8>(r);
                    r += dpp_d<kDppRor4>(r);
                    r = swap_add32(swap_add16(r));
                    const int wok = __all(okl);
                    if (lane < GB) s_cons[par][wave][q] = r;
                    if (lane == 0) s_cok[par][wave] = wok;
                    lds_barrier();
                    // flags and sums read together (one LDS round trip)
                    const int4 f = *reinterpret_cast<const int4*>(&s_cok[par][0]);
#pragma unroll
                    for (int u = 0; u < GB; ++u)
                        tot[u] = (s_cons[par][0][u] + s_cons[par][1][u]) +
                                 (s_cons[par][2][u] + s_cons[par][3][u]);
                    if (f.x && f.y && f.z && f.w) return true;
                    if (spins >= (kSpinLimit >> 4)) return false;   // uniform: every wave counts alike
                    lds_barrier();   // every wave has read this round's partials
                    __builtin_amdgcn_s_sleep(1);
                    poll_group(gc);
                }
            };
            // The loop is instantiated twice, with and without the stopping
            // test, so that neither carries the other's branches.
            auto run_groups = [&](auto check_tag) {
            constexpr bool CHECK = decltype(check_tag)::value;
            const int gend = CHECK ? glast + GLAG : glast;
            bool done = false;
            // momentum weights of the current group's steps; the next group's
            // are fetched a group ahead
            float bq[GB], bqn[GB];
#pragma unroll
            for (int u = 0; u < GB; ++u) bq[u] = a.beta[u];
            for (int gi = 1; gi <= gend && !done; ++gi) {
#pragma unroll
                for (int u = 0; u < GB; ++u) bqn[u] = a.beta[GB * gi + u];
#pragma unroll
                for (int u = 0; u < GB; ++u) {
                    const float beta = bq[u];
                    K = GB * (gi - 1) + 1 + u;
                    // Z_{K-1}, Z_{K-2} and their gradients
                    float (&z1)[TILES][NR] = (u == 0) ? sav[GB - 1] : cur[(u + GB - 1) % GB];
                    float (&z2)[TILES][NR] = (u == 0) ? sav[GB - 2] : (u == 1) ? sav[GB - 1] : cur[(u + GB - 2) % GB];
                    float (&g1)[TILES][NR] = gb2[(u + 1) & 1];
                    float (&g2)[TILES][NR] = gb2[u & 1];
                    const bool live = K <= kmax;   // later steps repeat Z_kmax
#pragma unroll
                    for (int t = 0; t < TILES; ++t)
#pragma unroll
                        for (int i = 0; i < NR; ++i) {
                            const float y = fmaf(beta, z1[t][i] - z2[t][i], z1[t][i]);
                            const float gy = fmaf(beta, g1[t][i] - g2[t][i], g1[t][i]);
                            const float v = fmaf(-gy, invL, y);
                            const float zn = (v > 0.f || v != v) ? v : 0.f;
                            cur[u][t][i] = live ? zn : z1[t][i];
                        }
                    double pv = 0.0;   // norm of step K - 1
#pragma unroll
                    for (int t = 0; t < TILES; ++t) pv += pg2_of(z1[t], g1[t]);
                    pgv[(u + GB - 1) % GB] = pv;
#pragma unroll
                    for (int t = 0; t < TILES; ++t) grad(cur[u][t], bb[t], g2[t]);
                    if constexpr (!CHECK) {
                        if (K == kmax) {
#pragma unroll
                            for (int t = 0; t < TILES; ++t)
#pragma unroll
                                for (int i = 0; i < NR; ++i) z[t][i] = cur[u][t][i];
                            steps = kmax;
                            done = true;
                            break;
                        }
                        continue;
                    } else {
                    if (u == 0 && gi >= 2) publish_group(gi - 1);
                    if (u == POLL_AT && testable(gi - GLAG)) poll_group(gi - GLAG);
                    if (u == TEST_AT && testable(gi - GLAG)) {
                        const int gc = gi - GLAG;
                        // iterates of the group under test
                        auto tz = [&](int uu, int t, int i) -> float {
                            if constexpr (GLAG > 1) return sav2[uu][t][i];
                            else return sav[uu][t][i];
                        };
                        double tot[GB];
                        if (!consume_group(gc, tot)) {
                            if (threadIdx.x == 0) raise_status(ctl, CNMF_ST_TIMEOUT);
                            ok = false;
                            done = true;
                            break;
                        }
                        // bit uu: step (gc - 1) GB + 1 + uu is testable and met the
                        // bound (hm) or has a non-finite norm (nm); every lane
                        // holds the same totals, so the masks are uniform
                        int hm = 0, nm = 0;
#pragma unroll
                        for (int uu = 0; uu < GB; ++uu) {
                            const int st = (gc - 1) * GB + 1 + uu;
                            const bool valid = st >= a.inner_min && st <= kmax;
                            hm |= (valid && tot[uu] <= tol2) ? (1 << uu) : 0;
                            nm |= (valid && !(tot[uu] == tot[uu])) ? (1 << uu) : 0;
                        }
                        hm = __builtin_amdgcn_readfirstlane(hm);
                        nm = __builtin_amdgcn_readfirstlane(nm);
                        const int hit = hm ? __builtin_ctz((unsigned)hm) : -1;
                        // non-finite norms at steps tested before the stop
                        if ((hit >= 0 ? nm & ((1 << hit) - 1) : nm) && blk == 0 && threadIdx.x == 0)
                            raise_status(ctl, CNMF_ST_NONFINITE);
                        if (hit >= 0) {
#pragma unroll
                            for (int uu = 0; uu < GB; ++uu)
                                if (uu == hit)
#pragma unroll
                                    for (int t = 0; t < TILES; ++t)
#pragma unroll
                                        for (int i = 0; i < NR; ++i) z[t][i] = tz(uu, t, i);
                            steps = (gc - 1) * GB + 1 + hit;
                            done = true;
                            break;
                        }
                        if (gc == glast) {   // budget spent without a stop: Z_kmax
#pragma unroll
                            for (int t = 0; t < TILES; ++t)
#pragma unroll
                                for (int i = 0; i < NR; ++i) z[t][i] = tz(GB - 1, t, i);
                            steps = kmax;
                            done = true;
                            break;
                        }
                    }
                    }   // CHECK
                }
                if (!done) {
#pragma unroll
                    for (int u = 0; u < GB; ++u) bq[u] = bqn[u];
#pragma unroll
                    for (int u = 0; u < GB; ++u)
#pragma unroll
                        for (int t = 0; t < TILES; ++t)
#pragma unroll
                            for (int i = 0; i < NR; ++i) {
                                if constexpr (GLAG > 1) sav2[u][t][i] = sav[u][t][i];
                                sav[u][t][i] = cur[u][t][i];
                            }
                }
            }
            if (!done && ok) {   // no group was testable: Z_kmax
#pragma unroll
                for (int t = 0; t < TILES; ++t)
#pragma unroll
                    for (int i = 0; i < NR; ++i) z[t][i] = sav[GB - 1][t][i];
                steps = kmax;
            }
            };
            if (check) run_groups(std::true_type{});
            else run_groups(std::false_type{});
        } else {
        // instantiated with and without the stopping test (as above)
        auto run_steps = [&](auto check_tag) {
        constexpr bool CHECK = decltype(check_tag)::value;
        kend = CHECK ? kmax + DLAG : kmax;
        float beta_n = a.beta[1];   // step K + 1, fetched a step ahead
        // restart: the step at which each row tile's momentum last restarted
        // (the start counts as a restart at step 1); row r's point Y_K uses
        // the weight of step K - k0 + 1 of a fresh loop
        int k0[TILES];
#pragma unroll
        for (int t = 0; t < TILES; ++t) k0[t] = 1;
        for (; K <= kend; ++K) {
            const int jst = K - DLAG;
            const bool test = CHECK && jst >= a.inner_min && jst <= kmax;
            // the poll of step K - DLAG is in flight during this step's compute
            if (test && wave == 0) poll_issue(jst, pwA);
            if (K <= kmax) {
                float zn[TILES][NR], gn[TILES][NR];
#pragma unroll
                for (int t = 0; t < TILES; ++t) {
                    float bt = beta;
                    if constexpr (RESTART) {
                        const int bi = K - k0[t];
                        bt = bi < kBetaLds ? sbeta[bi] : a.beta[bi];
                    }
                    float dr = 0.f;   // restart: (Y_K - Z_K) . (Z_K - Z_{K-1}) over the row
#pragma unroll
                    for (int i = 0; i < NR; ++i) {
                        const float y = fmaf(bt, zh[0][t][i] - zh[1][t][i], zh[0][t][i]);
                        const float gy = fmaf(bt, g[t][i] - gp[t][i], g[t][i]);
                        const float v = fmaf(-gy, invL, y);
                        zn[t][i] = (v > 0.f || v != v) ? v : 0.f;
                        if constexpr (RESTART) dr = fmaf(y - zn[t][i], zn[t][i] - zh[0][t][i], dr);
                    }
                    if constexpr (RESTART) {
                        if (row_sum4(dr) > 0.f) k0[t] = K;
                    }
                    grad(zn[t], bb[t], gn[t]);
                }
                beta = beta_n;
                beta_n = a.beta[K + 1];
#pragma unroll
                for (int j = NH - 1; j >= 1; --j)
#pragma unroll
                    for (int t = 0; t < TILES; ++t)
#pragma unroll
                        for (int i = 0; i < NR; ++i) zh[j][t][i] = zh[j - 1][t][i];
#pragma unroll
                for (int t = 0; t < TILES; ++t)
#pragma unroll
                    for (int i = 0; i < NR; ++i) {
                        zh[0][t][i] = zn[t][i];
                        gp[t][i] = g[t][i];
                        g[t][i] = gn[t][i];
                    }
                if (CHECK && K >= a.inner_min) {
                    double v = 0.0;
#pragma unroll
                    for (int t = 0; t < TILES; ++t) v += pg2_of(zh[0][t], g[t]);
                    publish(v, K);
                }
            } else {
                // past the budget: keep zh[j] = Z_{K-j} for the steps still to test
#pragma unroll
                for (int j = NH - 1; j >= 1; --j)
#pragma unroll
                    for (int t = 0; t < TILES; ++t)
#pragma unroll
                        for (int i = 0; i < NR; ++i) zh[j][t][i] = zh[j - 1][t][i];
            }
            if (test) {
                const double tot = collect(jst, true, pwA);
                if (s_flag) { ok = false; break; }
                if (!(tot == tot)) {
                    if (blk == 0 && threadIdx.x == 0) raise_status(ctl, CNMF_ST_NONFINITE);
                } else if (tot <= tol2) {
                    stop_at = jst;
                    break;
                }
            }
        }
        if (K > kend) K = kend;
        steps = stop_at >= 0 ? stop_at : kmax;
        out_idx = K - steps;   // 0 .. NH - 1
        };
        if (check) run_steps(std::true_type{});
        else run_steps(std::false_type{});
        }
    }
    }   // !ALT

    // final iterate zh[out_idx] -> z
#pragma unroll
    for (int j = 0; j < NH; ++j)
        if (j == out_idx)
#pragma unroll
            for (int t = 0; t < TILES; ++t)
#pragma unroll
                for (int i = 0; i < NR; ++i) z[t][i] = zh[j][t][i];

    // ---------------- 4. write back, next phase's partial product ----------
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
        const int64_t r = row_base + 16 * t + q16;
        if (r < a.rows && a.kind == 0) {
#pragma unroll
            for (int h = 0; h < PT; ++h)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int c = 16 * h + 4 * s + g4;
                    if (c < p) {
                        a.Z[r * a.z_rs + c * a.z_cs] = z[t][4 * h + s];
                        if (a.hist) a.hist[r * a.z_rs + c * a.z_cs] = z[t][4 * h + s];
                    }
                }
        }
    }
    if (a.part_out || a.part_out64) {
        // partial = sum over rows of q_r (x) z_r (mode 2, l x p) or z_r (x) z_r (p x p)
        constexpr int MT = 2;   // M tiles (l <= 32 or p <= 32)
        v4f acc[MT][PT];
#pragma unroll
        for (int hm = 0; hm < MT; ++hm)
#pragma unroll
            for (int hn = 0; hn < PT; ++hn) acc[hm][hn] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int h = 0; h < PT; ++h)
#pragma unroll
                for (int s = 0; s < 4; ++s) zt[wave][q16][16 * h + 4 * s + g4] = z[t][4 * h + s];
            if (PT == 1)
#pragma unroll
                for (int s = 0; s < 4; ++s) zt[wave][q16][16 + 4 * s + g4] = 0.f;
            // zt[wave] is this wave's own tile: no workgroup barrier (one
            // would also wait for the iterate's stores just issued)
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int rr = 4 * s + g4;                 // row within the tile (K index)
                const int64_t r = row_base + 16 * t + rr;
                float bv[PT];
#pragma unroll
                for (int hn = 0; hn < PT; ++hn) bv[hn] = zt[wave][rr][16 * hn + q16];
#pragma unroll
                for (int hm = 0; hm < MT; ++hm) {
                    float av;
                    if (a.mode == 2) {
                        const int k = 16 * hm + q16;
                        if constexpr (QPRE) av = qpre[t < (QPRE ? TILES : 1) ? t : 0][s][hm];
                        else av = (r < a.rows && k < a.ell) ? a.Q[r * a.ell + k] : 0.f;
                    } else {
                        av = (hm < PT) ? zt[wave][rr][16 * hm + q16] : 0.f;
                    }
#pragma unroll
                    for (int hn = 0; hn < PT; ++hn) acc[hm][hn] = mfma16(av, bv[hn], acc[hm][hn]);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        // reduce the 4 waves: element (M = 16 hm + 4 g4 + i, N = 16 hn + q16)
#pragma unroll
        for (int hm = 0; hm < MT; ++hm)
#pragma unroll
            for (int hn = 0; hn < PT; ++hn) settle(acc[hm][hn]);
#pragma unroll
        for (int hm = 0; hm < MT; ++hm)
#pragma unroll
            for (int hn = 0; hn < PT; ++hn)
#pragma unroll
                for (int i = 0; i < 4; ++i) sred[wave][(hm * 2 + hn) * 4 + i][lane] = acc[hm][hn][i];
        lds_barrier();
        for (int e = threadIdx.x; e < 16 * 64; e += kThreads) {
            const int ri = e / 64, l = e % 64;
            const int hm = (ri / 4) / 2, hn = (ri / 4) % 2, i = ri % 4;
            const int M = 16 * hm + 4 * (l >> 4) + i;
            const int N = 16 * hn + (l & 15);
            const float s = (sred[0][ri][l] + sred[1][ri][l]) + (sred[2][ri][l] + sred[3][ri][l]);
            const float v = hn < PT ? s : 0.f;
            // tagged words: only the entries the next phase polls (S is
            // l x p there); the plain layout is written whole
            if (a.part_out64) {
                if (M < (a.mode == 2 ? a.ell : 32) && N < p)
                    slot_store(&a.part_out64[(size_t)blk * 1024 + M * 32 + N], seq, __float_as_uint(v));
            } else {
                a.part_out[(size_t)blk * 1024 + M * 32 + N] = v;
            }
        }
    }

    if (threadIdx.x == 0) {
        if (blk == 0) {
            if (a.steps_out && a.kind == 0) a.steps_out[0] = steps;
            if (a.L_out) a.L_out[0] = L;
            if (a.tol_out) a.tol_out[0] = tol;
            if (a.pg2_out) a.pg2_out[0] = pg0;
            if (a.kind == 1 && a.tol_init_from) {
                const double tt = a.ratio * sqrt(pg0 + *a.tol_init_from);
                a.tol_init_out[0] = tt;
                a.tol_init_out[1] = tt;
                if (!isfinite(tt)) raise_status(ctl, CNMF_ST_NONFINITE);
            }
            if (!st && !ALT && a.kind == 0 && a.tol_state && steps >= 1 && steps <= a.inner_min)
                a.tol_state[0] = tol / 10.0;
            if (a.done_out) a.done_out[0] = a.done_value;
            if (a.deadline && a.stop_flag && wall_clock64() > *a.deadline) *a.stop_flag = 1;
            if (a.stop_word)
                slot_store(a.stop_word, seq, (a.deadline && wall_clock64() > *a.deadline) ? 1u : 0u);
        }
        if (a.tick_out) atomicMax(a.tick_out, (unsigned long long)wall_clock64());
    }
    // the running bound of the global rule: every workgroup took the same
    // decision with the same steps, so each keeps the same copy
    if (st && !ALT && a.kind == 0 && a.tol_state && steps >= 1 && steps <= a.inner_min)
        st->tol = tol / 10.0;
}

template <int PT, int TILES, int DLAG, int SOLVER = kSolverNesterov>
__global__ __launch_bounds__(kThreads) void k_phase(PhaseArgs a) {
    phase_body<PT, TILES, DLAG, SOLVER>(a, blockIdx.x, gridDim.x, a.seq);
}

template <int PT, int TILES, int DLAG, int SOLVER = kSolverNesterov>
hipError_t launch3(const Dev& d, const PhaseArgs& a, unsigned nblk) {
    hipLaunchKernelGGL((k_phase<PT, TILES, DLAG, SOLVER>), dim3(nblk), dim3(kThreads), 0, d.stream,
                       a);
    return hipGetLastError();
}

// Stop-test lag: -1 picks the grouped exchange when the iterate history
// fits the registers (PT * TILES <= 2), else a lag of two steps.  HALS and
// multiplicative updates test nothing; the restarted loop exchanges every
// step's norm, tested two steps late.
template <int PT, int TILES>
hipError_t launch2(const Dev& d, const PhaseArgs& a, unsigned nblk) {
    switch (a.solver) {
        case kSolverHals: return launch3<PT, TILES, 0, kSolverHals>(d, a, nblk);
        case kSolverMu: return launch3<PT, TILES, 0, kSolverMu>(d, a, nblk);
        case kSolverRestart: return launch3<PT, TILES, 2, kSolverRestart>(d, a, nblk);
        default: break;
    }
    int dl = a.dlag;
    if (dl < 0) dl = PT * TILES <= 2 ? kGrouped : 2;
    if (dl == kGrouped) {
        if constexpr (PT * TILES <= 2) return launch3<PT, TILES, kGrouped>(d, a, nblk);
        dl = 2;
    }
    switch (dl) {
        case 0: return launch3<PT, TILES, 0>(d, a, nblk);
        case 1: return launch3<PT, TILES, 1>(d, a, nblk);
        case 2: return launch3<PT, TILES, 2>(d, a, nblk);
        case 3: return launch3<PT, TILES, 3>(d, a, nblk);
        default: return launch3<PT, TILES, 4>(d, a, nblk);
    }
}

// The whole compressed outer loop in one launch (see LoopArgs): the G phase
// on workgroups < nbG, then the F phase on workgroups < nbF, T times.  The
// stop-test lag is the default one of each side's tile count.
// The arguments live in device memory and each phase reads its own copy
// after a compiler barrier: nothing of one phase's arguments stays live in
// scalar registers across the other phase.
template <int PT, int TG, int TF>
__global__ __launch_bounds__(kThreads) void k_phase_loop(const LoopArgs* __restrict__ Lp) {
    constexpr int DG = PT * TG <= 2 ? kGrouped : 2;
    constexpr int DF = PT * TF <= 2 ? kGrouped : 2;
    const unsigned blk = blockIdx.x;
    const int T = Lp->T;
    PhaseState sg{0.0, 0.0, 0.0}, sf{0.0, 0.0, 0.0};
    if (Lp->global_rule) {   // written by the launches before this one
        sg.tol = Lp->g.ctl->tol[0];
        sf.tol = Lp->g.ctl->tol[1];
    }
    for (int t = 0; t < T; ++t) {
        asm volatile("" ::: "memory");
        const LoopArgs& L = *Lp;
        const int p = L.g.p;
        if (blk < L.nbG) {
            PhaseArgs a = L.g;
            a.seq = L.seq0 + 2u * (unsigned)t;
            a.seq_in = t == 0 ? L.seq_pre : a.seq - 1u;
            if (a.forced_ptr) a.forced_ptr += 2 * t;
            if (a.steps_out) a.steps_out += 2 * t;
            if (a.L_out) a.L_out += 2 * t;
            if (a.tol_out) a.tol_out += 2 * t;
            if (a.hist) a.hist += (int64_t)t * L.g_hist_stride;
            if (a.w_out) a.w_out += (int64_t)(2 * t) * p * p;
            phase_body<PT, TG, DG>(a, blk, L.nbG, a.seq, &sg);
        }
        if (blk < L.nbF) {
            PhaseArgs a = L.f;
            a.seq = L.seq0 + 2u * (unsigned)t + 1u;
            a.seq_in = a.seq - 1u;
            if (a.forced_ptr) a.forced_ptr += 2 * t;
            if (a.steps_out) a.steps_out += 2 * t;
            if (a.L_out) a.L_out += 2 * t;
            if (a.tol_out) a.tol_out += 2 * t;
            if (a.hist) a.hist += (int64_t)t * L.f_hist_stride;
            if (a.w_out) a.w_out += (int64_t)(2 * t) * p * p;
            if (a.tick_out) a.tick_out += t;
            a.done_value = t + 1;
            asm volatile("" ::: "memory");
            phase_body<PT, TF, DF>(a, blk, L.nbF, a.seq, &sf);
        }
        if (L.f.stop_word) {
            // block 0's verdict after this outer iteration, the same for all
            // (thread 0 polls; the barrier hands the verdict to the others)
            const unsigned tag = L.seq0 + 2u * (unsigned)t + 1u;
            uint64_t w = 0;
            if (threadIdx.x == 0) {
                w = slot_load(L.f.stop_word);
                unsigned spins = 0;
                while ((unsigned)(w >> 32) != tag) {
                    __builtin_amdgcn_s_sleep(1);
                    if ((++spins & 255u) == 0u &&
                        (spins >= kSpinLimit || (atomic_status_load(&L.g.ctl->status) & CNMF_ST_TIMEOUT))) {
                        raise_status(L.g.ctl, CNMF_ST_TIMEOUT);
                        w = 1;   // leave
                        break;
                    }
                    w = slot_load(L.f.stop_word);
                }
            }
            if (__syncthreads_or((int)(w & 1u))) break;
        }
    }
}

template <int PT, int TG, int TF>
hipError_t launch_loop3(const Dev& d, const LoopArgs& a, const LoopArgs* dev_args) {
    const unsigned nb = a.nbG > a.nbF ? a.nbG : a.nbF;
    hipLaunchKernelGGL((k_phase_loop<PT, TG, TF>), dim3(nb), dim3(kThreads), 0, d.stream, dev_args);
    return hipGetLastError();
}

template <int PT>
hipError_t launch_loop(const Dev& d, const LoopArgs& a, const LoopArgs* da, int tg, int tf) {
    if (tg == 1) return tf == 1 ? launch_loop3<PT, 1, 1>(d, a, da) : launch_loop3<PT, 1, 2>(d, a, da);
    return tf == 1 ? launch_loop3<PT, 2, 1>(d, a, da) : launch_loop3<PT, 2, 2>(d, a, da);
}

template <int PT>
hipError_t launch1(const Dev& d, const PhaseArgs& a, int tiles, unsigned nblk) {
    switch (tiles) {
        case 1: return launch2<PT, 1>(d, a, nblk);
        case 2: return launch2<PT, 2>(d, a, nblk);
        default: return launch2<PT, 4>(d, a, nblk);
    }
}

// Batched form: many subproblems in one persistent launch.  Workgroup s
// walks the rounds of a schedule; in round r it solves the subproblem and
// part named by sched[r][s] (instance << 12 | block), or idles.  All blocks
// of a subproblem sit in the same round, and every workgroup is resident,
// so the workgroups a subproblem waits for are always running or will reach
// it.  The launch tag comes from device memory (*epoch) and the last
// workgroup to finish advances it, so a captured graph can replay the
// launch; when the tag wraps, that workgroup clears every instance's
// exchange words first.
template <int TILES, int DLAG>
__global__ __launch_bounds__(kThreads) void k_phase_batched(BatchLaunch b) {
    __shared__ unsigned s_last;
    const unsigned seq = *b.epoch;
    for (int r = 0; r < b.rounds; ++r) {
        const uint32_t e = b.sched[(size_t)r * gridDim.x + blockIdx.x];
        if (e == 0xffffffffu) continue;
        const PhaseArgs& a = b.args[e >> 12];
        if (a.p <= 16) phase_body<1, TILES, DLAG>(a, e & 0xfffu, a.nblk, seq);
        else phase_body<2, TILES, DLAG>(a, e & 0xfffu, a.nblk, seq);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned old = atomicAdd(b.done, 1u);
        s_last = old == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last) {
        const unsigned nx = seq + 1 < (1u << 22) ? seq + 1 : 1u;
        if (nx == 1u) {
            for (int i = 0; i < b.count; ++i) {
                uint64_t* w = b.args[i].slot_s;
                for (size_t k = threadIdx.x; k < kSlotWords; k += kThreads) w[k] = 0;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            *b.done = 0;
            *b.epoch = nx;
        }
    }
}

template <int TILES>
hipError_t launch_batched2(const Dev& d, const BatchLaunch& b, int dlag) {
    dim3 grid((unsigned)b.slots), block(kThreads);
    if (dlag < 0) dlag = TILES == 1 ? kGrouped : 2;
    if (dlag == kGrouped) {
        if constexpr (TILES == 1) {
            hipLaunchKernelGGL((k_phase_batched<1, kGrouped>), grid, block, 0, d.stream, b);
            return hipGetLastError();
        }
        dlag = 2;
    }
    switch (dlag) {
        case 0: hipLaunchKernelGGL((k_phase_batched<TILES, 0>), grid, block, 0, d.stream, b); break;
        case 1: hipLaunchKernelGGL((k_phase_batched<TILES, 1>), grid, block, 0, d.stream, b); break;
        case 2: hipLaunchKernelGGL((k_phase_batched<TILES, 2>), grid, block, 0, d.stream, b); break;
        case 3: hipLaunchKernelGGL((k_phase_batched<TILES, 3>), grid, block, 0, d.stream, b); break;
        default: hipLaunchKernelGGL((k_phase_batched<TILES, 4>), grid, block, 0, d.stream, b); break;
    }
    return hipGetLastError();
}

}  // namespace

// Rows per workgroup and grid for `rows` rows: the grid must fit on the CUs
// at once (workgroups wait for each other's partial norms).
bool phase_grid(const Dev& d, int64_t rows, int* tiles, unsigned* nblk) {
    for (int t : {1, 2, 4}) {
        const int64_t nb = (rows + 64 * t - 1) / (64 * t);
        if (nb <= d.num_cus && nb <= 256) {
            *tiles = t;
            *nblk = (unsigned)(nb < 1 ? 1 : nb);
            return true;
        }
    }
    return false;
}

hipError_t phase_batched(const Dev& d, const BatchLaunch& b, int tiles, int dlag) {
    if (dlag < -1 || (dlag > 4 && dlag != kGrouped) || b.slots < 1) return hipErrorInvalidValue;
    switch (tiles) {
        case 1: return launch_batched2<1>(d, b, dlag);
        case 2: return launch_batched2<2>(d, b, dlag);
        default: return launch_batched2<4>(d, b, dlag);
    }
}

bool phase_loop_supported(int p, int tilesG, int tilesF) {
    return p >= 1 && p <= 32 && (tilesG == 1 || tilesG == 2) && (tilesF == 1 || tilesF == 2);
}

hipError_t phase_loop(const Dev& d, const LoopArgs& a, LoopArgs* dev_args, int tilesG, int tilesF) {
    if (!phase_loop_supported(a.g.p, tilesG, tilesF) || a.T < 1 || a.g.mode != 2 || a.f.mode != 2 ||
        a.g.solver != kSolverNesterov || a.f.solver != kSolverNesterov || !a.g.part_in64 ||
        !a.g.part_out64 || !a.f.part_in64 || !a.f.part_out64 || a.g.stop_flag || a.f.stop_flag ||
        a.g.stop_word || (a.f.stop_word && !a.f.deadline))
        return hipErrorInvalidValue;
    // the argument block goes to device memory ahead of the launch (a copy
    // from pageable memory returns once the source has been read)
    hipError_t e = hipMemcpyAsync(dev_args, &a, sizeof(LoopArgs), hipMemcpyHostToDevice, d.stream);
    if (e != hipSuccess) return e;
    if (a.g.p <= 16) return launch_loop<1>(d, a, dev_args, tilesG, tilesF);
    return launch_loop<2>(d, a, dev_args, tilesG, tilesF);
}

hipError_t phase(const Dev& d, const PhaseArgs& a, unsigned nblk, int tiles) {
    if (a.p < 1 || a.p > 32 || a.dlag < -1 || (a.dlag > 4 && a.dlag != kGrouped))
        return hipErrorInvalidValue;
    if (a.solver < kSolverNesterov || a.solver > kSolverRestart) return hipErrorInvalidValue;
    if (a.p <= 16) return launch1<1>(d, a, tiles, nblk);
    return launch1<2>(d, a, tiles, nblk);
}

// lambda_max of a p x p FP32 matrix, one wavefront (kernel-level entry point).
namespace {
__global__ __launch_bounds__(64) void k_lips(int p, const float* __restrict__ W,
                                             double* __restrict__ out, Control* ctl) {
    __shared__ double A[32][33];
    __shared__ double v[32], wv[32], dg[32], eo[32];
    for (int e = threadIdx.x; e < p * p; e += 64) {
        const int i = e / p, j = e % p;
        A[i][j] = 0.5 * ((double)W[i * p + j] + (double)W[j * p + i]);
    }
    __syncthreads();
    const double lm = lambda_max_wave(A, p, v, wv, dg, eo);
    if (threadIdx.x == 0) {
        out[0] = lm;
        if (lm != lm) raise_status(ctl, CNMF_ST_NONFINITE);
    }
}
}  // namespace

hipError_t lipschitz(const Dev& d, int p, const float* W, double* out, Control* ctl) {
    hipLaunchKernelGGL(k_lips, dim3(1), dim3(64), 0, d.stream, p, W, out, ctl);
    return hipGetLastError();
}

}  // namespace cnmf
