// Internal declarations shared by the HIP translation units of libcnmf.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cnmf.h"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

namespace cnmf {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Device-side control block, one per context (device memory, zeroed at
// creation).  Grid barriers of the persistent kernels live here.
// ---------------------------------------------------------------------------
struct Control {
    unsigned bar_count;   // arrivals at the current grid barrier
    unsigned bar_gen;     // barrier generation, grows forever
    int status;           // CNMF_ST_* bits
    int pad0;
    double pg2[4];        // scratch for initial projected-gradient norms
    double tol[2];        // running gradient bounds (G, F) of the global rule
    unsigned long long deadline;   // wall clock at which a time-budgeted outer loop stops
    int stop;             // set once the deadline has passed: later phases do nothing
    int pad1;
};

// Spin limit of a grid barrier: about a second of polling before the
// barrier gives up, flags CNMF_ST_TIMEOUT and lets every wave leave.
constexpr unsigned kSpinLimit = 1u << 24;

__device__ __forceinline__ int atomic_status_load(int* s) {
    return __hip_atomic_load(s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void raise_status(Control* ctl, int bits) {
    __hip_atomic_fetch_or(&ctl->status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sense-free generation barrier across all workgroups of a grid whose
// workgroups are all resident (grid size <= number of CUs).  Every thread
// of every workgroup must call it.  Returns false when the barrier timed
// out or a timeout was already flagged; callers then leave their loops.
__device__ __forceinline__ bool grid_sync(Control* ctl, unsigned nblocks) {
    __shared__ int s_ok;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned g = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned a = __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL,
                                            __HIP_MEMORY_SCOPE_AGENT);
        if (a == nblocks - 1) {
            __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&ctl->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                if (((++spins) & 1023u) == 0u) {
                    if (spins >= kSpinLimit || (atomic_status_load(&ctl->status) & CNMF_ST_TIMEOUT)) {
                        raise_status(ctl, CNMF_ST_TIMEOUT);
                        ok = 0;
                        break;
                    }
                }
            }
        }
        if (atomic_status_load(&ctl->status) & CNMF_ST_TIMEOUT) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    __threadfence();
    return s_ok != 0;
}

// Wavefront reductions with DPP row operations (no LDS traffic): xor 1 and
// xor 2 inside quads, rotations by 4 and 8 inside 16-lane rows, then the four
// row results combined in a fixed order.  Every lane gets the same value and
// the result is bit-identical across runs and across workgroups.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppRor4 = 0x124;    // row_ror:4
constexpr int kDppRor8 = 0x128;    // row_ror:8

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<kDppXor1>(v);
    v += dpp_d<kDppXor2>(v);
    v += dpp_d<kDppRor4>(v);
    v += dpp_d<kDppRor8>(v);
    return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// Pairwise sums across 16-lane rows (rows 0+1 and 2+3) and across the two
// 32-lane halves, by the row and half swaps: both lanes of a pair add the
// same two operands in the same order, so they hold the same bits.
__device__ __forceinline__ double swap_add16(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    const double y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
    return x + y;
}
__device__ __forceinline__ double swap_add32(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    const double y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
    return x + y;
}

// Four wavefront sums at once: lane L returns the total over the wavefront of
// v[quad_slot(L)].  Quad exchanges leave one partial of each of the four
// values per quad, row rotations by 8 then 4 and the row and half swaps
// finish the sum; each step adds two operands that the partner lane adds in
// the same or the other order, so all lanes with the same slot hold the same
// bits.
__device__ __forceinline__ int quad_slot(int lane) { return 2 * (lane & 1) + ((lane >> 1) & 1); }
__device__ __forceinline__ double wave_sum4(const double (&v)[4]) {
    const int lane = threadIdx.x & 63;
    const bool odd = lane & 1;
    const double a0 = (odd ? v[2] : v[0]) + dpp_d<kDppXor1>(odd ? v[0] : v[2]);
    const double a1 = (odd ? v[3] : v[1]) + dpp_d<kDppXor1>(odd ? v[1] : v[3]);
    const bool hi = (lane >> 1) & 1;
    double b = (hi ? a1 : a0) + dpp_d<kDppXor2>(hi ? a0 : a1);
    b += dpp_d<kDppRor8>(b);
    b += dpp_d<kDppRor4>(b);
    return swap_add32(swap_add16(b));
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<kDppXor1>(v);
    v += dpp_f<kDppXor2>(v);
    v += dpp_f<kDppRor4>(v);
    v += dpp_f<kDppRor8>(v);
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (a + b) + (c + d);
}

__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<kDppXor1>(v));
    v = fmax(v, dpp_d<kDppXor2>(v));
    v = fmax(v, dpp_d<kDppRor4>(v));
    v = fmax(v, dpp_d<kDppRor8>(v));
    return fmax(fmax(lane_d(v, 0), lane_d(v, 16)), fmax(lane_d(v, 32), lane_d(v, 48)));
}

// FP32 -> bfloat16 bits, round to nearest even; NaN stays NaN (quiet).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint32_t rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const uint32_t quiet = (u >> 16) | 0x40u;
    return (uint16_t)(((u & 0x7fffffffu) > 0x7f800000u) ? quiet : rounded);   // select, no branch
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (defined in the .hip files, called by api.cpp).
// All return hipSuccess or the launch error.
// ---------------------------------------------------------------------------
struct Dev {
    int device;
    int num_cus;
    hipStream_t stream;
};

// sweep.hip
size_t sweep_right_partial_floats(const Dev& d, int64_t R, int64_t C);
hipError_t sweep_right(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx,
                       int k, const float* A, int64_t lda, bool a_trans, float* Y,
                       int64_t ldy, float* partial);
size_t sweep_left_partial_floats(const Dev& d, int64_t R, int64_t C);
hipError_t sweep_left(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx,
                      int k, const float* B, int64_t ldb, float* Z, int64_t ldz,
                      bool z_trans, float* partial);
// sweep_dual.hip: Y (R x k, ldy) = X A with A given as its transpose AT
// (k x C, ldat) and Z = X^T B (B R x k, ldb; Z C x k, or k x C if z_trans)
// from one read of X; FP32 accuracy from three-way BF16 splits on the
// matrix cores, k <= 32 (hipErrorInvalidValue beyond).
size_t sweep_dual_partial_floats(const Dev& d, int64_t R, int64_t C);
hipError_t sweep_dual(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx, int k,
                      const float* AT, int64_t ldat, const float* B, int64_t ldb, float* Y,
                      int64_t ldy, float* Z, int64_t ldz, bool z_trans, float* partial);
// The same pair with X in bfloat16 (Xb, row pitch ldx in elements), both
// skinny operands rounded to bfloat16, FP32 accumulation; partial: workspace
// of sweep_dual_bf16_partial_floats(d, R, C) floats.
size_t sweep_dual_bf16_partial_floats(const Dev& d, int64_t R, int64_t C);
hipError_t sweep_dual_bf16(const Dev& d, int64_t R, int64_t C, const uint16_t* Xb, int64_t ldx,
                           int k, const float* AT, int64_t ldat, const float* B, int64_t ldb,
                           float* Y, int64_t ldy, float* Z, int64_t ldz, bool z_trans,
                           float* partial);
// Batched sweeps: one descriptor per instance; work items {instance, item}
// with item = slice * tiles + tile (sweeps), a 256-element chunk of the
// slice reduction, or a 32 x 32 transpose tile.  X rows and the skinny
// operands must allow 16-byte vector loads (row pitches multiple of 4).
struct SweepDesc {
    int64_t R, C;          // X is R x C
    const float* X;
    int64_t ldx;
    int k, nt;             // columns of the skinny operand, MFMA tile width (16 / 32)
    const float* A;        // right: A^T (k x C, lda); left: B (R x k, lda)
    int64_t lda;
    float* partial;        // [S][rows][nt], rows = R (right) or C (left)
    int64_t span;          // right: columns per slice; left: rows per slice
    int tiles, S;
    float* Y;              // reduction output (rows x k, or k x rows when trans)
    int64_t ldy;
    int trans;
};
struct WorkItem {
    int inst, item;
};
// Plans: tiles and slices for one instance (S = 1 unless `slices` > 1).
void sweep_desc_right(SweepDesc* s, int64_t R, int64_t C, const float* X, int64_t ldx, int k,
                      const float* AT, int64_t ldt, float* partial, float* Y, int64_t ldy);
void sweep_desc_left(SweepDesc* s, int64_t R, int64_t C, const float* X, int64_t ldx, int k,
                     const float* B, int64_t ldb, float* partial, float* Y, int64_t ldy,
                     bool trans);
hipError_t sweep_right_batched(const Dev& d, const SweepDesc* desc, const WorkItem* work,
                               int64_t nwork);
hipError_t sweep_left_batched(const Dev& d, const SweepDesc* desc, const WorkItem* work,
                              int64_t nwork);
hipError_t reduce_batched(const Dev& d, const SweepDesc* desc, const WorkItem* work,
                          int64_t nwork, bool left);
// out (B: C x R, ldb) = A^T for every descriptor {R, C, A, lda, B, ldb}.
struct TransDesc {
    int64_t R, C;
    const float* A;
    int64_t lda;
    float* B;
    int64_t ldb;
};
hipError_t transpose_batched(const Dev& d, const TransDesc* desc, const WorkItem* work,
                             int64_t nwork);

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations (lgkmcnt) but not for its outstanding global loads, so loads
// issued earlier (a poll of exchange words, the next tile of a stream) stay
// in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // vmcnt / expcnt untouched, lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
}

// reduce_slices: out (rows x k, or k x rows if trans) = sum of S partial
// slices [S][rows][nt] in slice order (bitwise reproducible).
hipError_t reduce_slices(const Dev& d, int64_t rows, int k, int64_t S, int nt,
                         const float* partial, float* out, int64_t ldo, bool trans);
// Workgroups per slice so that one round of the grid fills every CU.
inline int64_t pick_splits(int64_t tiles, int64_t kunits, int num_cus, int occ) {
    const int64_t slots = (int64_t)num_cus * (occ > 0 ? occ : 1);
    int64_t S = slots / tiles;
    if (S > kunits) S = kunits;
    if (S < 1) S = 1;
    return S;
}

// sweep_bf16.hip: the same products with X in bfloat16 (and the skinny
// operand rounded to bfloat16), FP32 accumulation on the matrix cores.
// pack: workspace of bf16_pack_elems(C) 16-bit words for the right sweep's
// rounded panel.
size_t bf16_pack_elems(int64_t C);
size_t sweep_right_bf16_partial_floats(const Dev& d, int64_t R, int64_t C);
hipError_t sweep_right_bf16(const Dev& d, int64_t R, int64_t C, const uint16_t* Xb,
                            int64_t ldx, int k, const float* A, int64_t lda, bool a_trans,
                            float* Y, int64_t ldy, float* partial, uint16_t* pack);
size_t sweep_left_bf16_partial_floats(const Dev& d, int64_t R, int64_t C);
hipError_t sweep_left_bf16(const Dev& d, int64_t R, int64_t C, const uint16_t* Xb,
                           int64_t ldx, int k, const float* B, int64_t ldb, float* Z,
                           int64_t ldz, bool z_trans, float* partial);
hipError_t to_bf16(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx,
                   uint16_t* Xb, int64_t ldxb);
hipError_t transpose(const Dev& d, int64_t R, int64_t C, const float* A, int64_t lda,
                     float* B, int64_t ldb);
hipError_t check_input(const Dev& d, int64_t R, int64_t C, const float* X, int64_t ldx,
                       Control* ctl);

// orth.hip: CholeskyQR (second pass when ill-conditioned) with the rank rule
// in one launch.  xch: exchange
// words (orth_exchange_words(), room for two panels at once; a single panel
// uses the first half); seq: launch tag (< 2^22), fresh per call.
// QT (optional): transposed copy of Q with row pitch ldqt.
size_t orth_exchange_words();

constexpr int kOrthMaxPairs = 64 * 65 / 2;   // entries of the largest (augmented) Gram
// Arguments of one panel's orthonormalisation (batched launches keep an
// array of them on the device).
struct OrthArgs {
    int64_t N;
    int l;
    const float* Y;
    const float* P;
    int64_t p_rs, p_cs;
    double tau2;
    float* Q;           // N x l
    float* QT;          // optional l x N copy, row pitch ldqt
    int64_t ldqt;
    int32_t* replaced;  // optional l flags
    uint64_t* part;     // [nblk][kMaxPairs][2]
    uint64_t* red;      // [kMaxPairs][2]
    unsigned seq;
    Control* ctl;
    unsigned nblk;      // batched launches: workgroups of this panel
};

// Batched orthonormalisation: exchange words per panel, workgroups per
// panel, argument helper and the launch over a round schedule (as for the
// batched subproblems).
size_t orth_batch_exchange_words(unsigned nblk);
unsigned orth_batch_blocks(int64_t N);
OrthArgs orth_args(int64_t N, int l, const float* Y, const float* pool, bool pool_trans,
                   double tau2, float* Q, float* QT, int64_t ldqt, int32_t* replaced,
                   uint64_t* xch, unsigned seq, Control* ctl, unsigned nblk);
hipError_t orth_batched(const Dev& d, const OrthArgs* args, const uint32_t* sched, int rounds,
                        int slots);
hipError_t orth(const Dev& d, int64_t N, int l, const float* Y, const float* pool,
                bool pool_trans, double tau2, float* Q, float* QT, int64_t ldqt,
                int32_t* replaced, uint64_t* xch, unsigned seq, Control* ctl);
// Two independent panels in one launch (half of the workgroups each), so
// their exchange latencies overlap; a and b come from orth_args() with xch
// set to the two halves of the context's exchange words and fresh tags.
hipError_t orth_pair(const Dev& d, OrthArgs a, OrthArgs b);
unsigned orth_pair_blocks(const Dev& d, int64_t N);

// small.hip
hipError_t lipschitz(const Dev& d, int p, const float* W, double* out, Control* ctl);

// solver.hip
// Kernel arguments of one phase.
struct PhaseArgs {
    int64_t rows;
    int p;
    int ell;                 // compressed: l; plain / given: 0
    int mode;                // 0 given W/B, 1 plain (W from partials, B given), 2 compressed
    int wt;                  // 1: gradient Z W^T (F update in row form)
    float* Z;
    int64_t z_rs, z_cs;
    const float* Bgiven;     // rows x p (modes 0, 1)
    const float* Wgiven;     // p x p (mode 0)
    const float* D;          // compressed data, element (r, k) at D[r*d_rs + k*d_cs]
    int64_t d_rs, d_cs;
    const float* Q;          // rows x l, row-major (mode 2 epilogue)
    const float* part_in;    // [nin][32][32] partial products of the previous phase
    int nin;
    float* part_out;         // [nblk][32][32] (may be null)
    uint64_t* slot_s;        // [1024] S exchange
    uint64_t* slot_pg;       // kPgWords projected-gradient exchange words
    const float* beta;       // momentum weight of inner step K at beta[K - 1] (kBetaLen)
    unsigned seq;            // launch sequence (tag), 1 .. 2^22 - 1
    Control* ctl;
    // stopping
    const double* tol_ptr;   // global rule: running bound (read)
    double* tol_state;       // global rule: divided by 10 after an early stop
    double tol_value;        // given bound (mode 0 without tol_ptr)
    double ratio;            // > 0: per-subproblem rule
    int inner_max, inner_min, forced;
    const int32_t* forced_ptr;
    int dlag;
    // outputs
    int32_t* steps_out;
    double* L_out;
    double* tol_out;
    double* pg2_out;         // ||P grad(Z_0)||^2
    int kind;                // 0 solve, 1 projected-gradient norm only, 2 partial product only
    double* tol_init_from;   // with kind 1: tol = ratio*sqrt(pg2 + *tol_init_from) -> tol_init_out[0..1]
    double* tol_init_out;
    unsigned nblk;           // workgroups of this subproblem (batched launches)
    const double* eig_in;    // {L, v[32]} of the previous subproblem of this side, or null
    double* eig_out;         // {L, v[32]} of this subproblem (written by block 0), or null
    float* hist;
    unsigned long long* tick_out;
    float* w_out;            // p x p: W as used by this subproblem (block 0), or null
    // time budget: a phase does nothing once *stop_flag is set; block 0 of a
    // phase with done_out writes done_value there when it completes and, with
    // deadline, sets *stop_flag when the wall clock has passed *deadline
    int* stop_flag;
    int32_t* done_out;
    int done_value;
    const unsigned long long* deadline;
    int solver;              // kSolver*: update rule of the subproblem
    // partial products as tagged words {seq : 32 | FP32 bits : 32} instead of
    // part_in / part_out, for phases that follow each other inside one launch
    // (the fused outer loop): a reader polls each word until it carries the
    // writer's tag, so no kernel boundary is needed between the phases
    const uint64_t* part_in64;   // [nin][32][32], written with tag seq_in
    unsigned seq_in;
    uint64_t* part_out64;        // [nblk][32][32], written with tag seq
    // fused loop with a time budget: block 0 publishes here, tagged with seq,
    // whether the wall clock has passed *deadline (1) or not (0)
    uint64_t* stop_word;
};

// Whole compressed outer loop in one launch (Algorithm 1 with the Nesterov
// inner loop of Sec. 2): for t < T, the G phase on workgroups < nbG, then the
// F phase on workgroups < nbF.  g and f are the phases' arguments at t = 0;
// the per-iteration outputs advance by their strides, the replayed step
// counts by 2 per iteration, and the tags are seq0 + 2 t (G) and
// seq0 + 2 t + 1 (F); the first G phase reads F's partials written with tag
// seq_pre.  Every workgroup keeps the warm start of lambda_max and the
// running bound of the global rule itself (every workgroup computes the
// same values), so the partial products are the only data that cross
// workgroups between phases.  With f.stop_word (a time budget), every
// workgroup reads block 0's verdict after each F phase and all leave the
// loop after the same outer iteration.
struct LoopArgs {
    PhaseArgs g, f;
    int T;
    unsigned nbG, nbF;
    unsigned seq0, seq_pre;
    int64_t g_hist_stride, f_hist_stride;   // floats per outer iteration
    int global_rule;                        // running bounds start from ctl->tol
};
hipError_t phase_loop(const Dev& d, const LoopArgs& a, LoopArgs* dev_args, int tilesG,
                      int tilesF);   // dev_args: device memory for one LoopArgs
bool phase_loop_supported(int p, int tilesG, int tilesF);

// Batched launch of many subproblems (see k_phase_batched): args[count] on
// the device, sched[rounds][slots] entries (instance << 12 | block) or
// 0xffffffff; epoch / done: device words owned by the batch.
struct BatchLaunch {
    const PhaseArgs* args;
    const uint32_t* sched;
    int count;
    int rounds;
    int slots;
    unsigned* epoch;
    unsigned* done;
};
hipError_t phase_batched(const Dev& d, const BatchLaunch& b, int tiles, int dlag);

bool phase_grid(const Dev& d, int64_t rows, int* tiles, unsigned* nblk);
hipError_t phase(const Dev& d, const PhaseArgs& a, unsigned nblk, int tiles);
constexpr int kPgSlots = 10;   // slots per workgroup for projected-gradient partials
constexpr size_t kPgWords = 8192;   // projected-gradient exchange words
// Momentum weights of the inner loop (Sec. 2): alpha_0 = 1,
// alpha_{k+1} = (1 + sqrt(4 alpha_k^2 + 1)) / 2, and inner step K uses
// beta = (alpha_{K-2} - 1) / alpha_{K-1} (0 for K <= 2), rounded to FP32.  They
// depend on K alone, so one table (host-made, FP64 recursion) serves every
// launch; it covers the largest inner budget plus the steps a stop test lags.
constexpr int kBetaLen = 100000 + 64;
inline void momentum_table(float* out, int n) {
    double alpha = 1.0;
    float beta = 0.f;
    for (int k = 0; k < n; ++k) {
        out[k] = beta;
        const double alpha_n = 0.5 * (1.0 + std::sqrt(std::fma(4.0 * alpha, alpha, 1.0)));
        beta = (float)((alpha - 1.0) / alpha_n);
        alpha = alpha_n;
    }
}
constexpr size_t kSlotWords = 1024 + kPgWords;
// Update rules of a phase (PhaseArgs::solver): the Nesterov loop of Sec. 2,
// the same with adaptive restart, HALS sweeps, multiplicative updates.
constexpr int kSolverNesterov = 0;
constexpr int kSolverHals = 1;
constexpr int kSolverMu = 2;
constexpr int kSolverRestart = 3;
constexpr int kBetaLds = 1024;   // momentum weights a restarted loop keeps in LDS
constexpr int kGrouped = 8;     // stop-test lag value selecting the grouped exchange
constexpr int kEigWords = 33;   // {L, v[32]} per side and parity

// misc kernels (small.hip)
hipError_t write_tick(const Dev& d, unsigned long long* tick);
// ctl->deadline = now + ticks, ctl->stop = 0 (start of a time-budgeted loop)
hipError_t arm_deadline(const Dev& d, Control* ctl, unsigned long long ticks);
hipError_t fill_u64(const Dev& d, uint64_t* p, int64_t count, uint64_t value);
hipError_t fill_i32(const Dev& d, int32_t* p, int64_t count, int32_t value);
// dst = scale * src over a rows x cols block (src may be dst)
hipError_t scale2d(const Dev& d, int64_t rows, int64_t cols, const float* src, int64_t lds,
                   float* dst, int64_t ldd, float scale);
// A /= ||A||_F (FP64 sum of squares; part: kNormBlocks doubles of scratch)
constexpr int kNormBlocks = 256;
hipError_t normalize2d(const Dev& d, int64_t rows, int64_t cols, float* A, int64_t lda,
                       double* part);
hipError_t rre(const Dev& d, int64_t n, int64_t m, const float* X, int64_t ldx, int p,
               const float* G, int64_t sG, const float* F, int64_t sF, int count,
               double* out, double* partial, int64_t partial_len);
size_t rre_partial_doubles(const Dev& d, int64_t n, int64_t m, int count);

}  // namespace cnmf
