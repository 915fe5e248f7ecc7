// NeNMF inner loop (Sec. 2) as one persistent kernel.
//
// Problem: min_{Z >= 0} 0.5 tr(Z W Z^T) - tr(B^T Z) over `rows` rows of p
// unknowns (G update of Eq. (2): Z = G, W = F F^T, B = X F^T; F update of
// Eq. (3) by columns: Z = F^T, W = G^T G, B = (G^T X)^T; compressed forms of
// Algorithm 1 with F_R, G_L, X_R, X_L).  Rows are independent except for the
// stopping test, a bound on the Frobenius norm of the projected gradient of
// the whole factor.
//
// Step k (alpha_0 = 1, Y_1 = Z_0):
//   Z_k     = max(0, Y_k - grad(Y_k) / L)
//   alpha_k = (1 + sqrt(4 alpha_{k-1}^2 + 1)) / 2
//   Y_{k+1} = Z_k + ((alpha_{k-1} - 1) / alpha_k) (Z_k - Z_{k-1})
// and stop at the first k >= inner_min with ||P grad(Z_k)||_F <= tol.
//
// One thread owns one row: Z_k, Z_{k-1}, grad(Z_k), grad(Z_{k-1}) and B stay
// in registers, W in LDS.  Only grad(Z_k) is formed by a product with W;
// grad(Y_{k+1}) follows by linearity from the last two gradients.  The
// squared norm of the projected gradient is summed in FP64: wave butterfly,
// LDS across the workgroup, then one partial per workgroup read back by
// every workgroup after a grid barrier and summed in the same order, so all
// workgroups take the same stop decision.
#include "internal.hpp"

namespace cnmf {

namespace {

constexpr int kThreads = 256;

struct KArgs {
    int64_t rows;
    float* Z;
    int64_t z_rs, z_cs;
    const float* W;
    const float* B;
    const double* L;
    const double* tol_ptr;
    double tol_value;
    double ratio;
    double* tol_state;
    int inner_max, inner_min;
    int forced;
    const int32_t* forced_ptr;
    int32_t* steps_out;
    double* L_out;
    double* tol_out;
    double* pg2_out;
    float* hist;
    unsigned long long* tick_out;
    int pg_only;
};

// Sum of one double per thread over the whole grid; identical in every
// workgroup.  `slot` alternates so that a fast workgroup never overwrites
// partials a slow one has yet to read.
__device__ __forceinline__ double grid_total(double v, double* partials, int slot,
                                             Control* ctl, unsigned nblk, bool& ok,
                                             double* s_red, double* s_tot) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        partials[(size_t)slot * nblk + blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
    ok = grid_sync(ctl, nblk) && ok;
    if (wave == 0) {
        double t = 0.0;
        for (unsigned i = lane; i < nblk; i += 64) t += partials[(size_t)slot * nblk + i];
        t = wave_sum(t);
        if (lane == 0) *s_tot = t;
    }
    __syncthreads();
    return *s_tot;
}

template <int P>
__device__ __forceinline__ void matvec(const float* __restrict__ sW, const float (&z)[P],
                                       const float (&b)[P], float (&g)[P]) {
#pragma unroll
    for (int c = 0; c < P; ++c) g[c] = -b[c];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const float zi = z[i];
#pragma unroll
        for (int c = 0; c < P; ++c) g[c] = fmaf(zi, sW[i * P + c], g[c]);
    }
}

template <int P>
__device__ __forceinline__ double pg2_row(const float (&z)[P], const float (&g)[P]) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        const float pg = (z[c] > 0.f) ? g[c] : fminf(g[c], 0.f);
        // keep NaN visible: fminf drops it, so test explicitly
        const double d = (g[c] != g[c]) ? (double)g[c] : (double)pg;
        s = fma(d, d, s);
    }
    return s;
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_nnls(KArgs a, double* partials, Control* ctl) {
    __shared__ float sW[P * P];
    __shared__ double s_red[4];
    __shared__ double s_tot;
    const unsigned nblk = gridDim.x;
    for (int e = threadIdx.x; e < P * P; e += kThreads) sW[e] = a.W[e];
    __syncthreads();

    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool active = r < a.rows;
    float* zrow = a.Z + (active ? r : 0) * a.z_rs;
    float z[P], b[P], g[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        z[c] = active ? zrow[c * a.z_cs] : 0.f;
        b[c] = active ? a.B[(active ? r : 0) * P + c] : 0.f;
    }
    matvec<P>(sW, z, b, g);
    bool ok = true;

    const double L = a.pg_only ? 1.0 : *a.L;
    const bool need_pg0 = a.pg_only || a.pg2_out != nullptr || a.ratio > 0.0;
    double pg0 = 0.0;
    if (need_pg0) {
        pg0 = grid_total(active ? pg2_row<P>(z, g) : 0.0, partials, 0, ctl, nblk, ok, s_red, &s_tot);
        if (blockIdx.x == 0 && threadIdx.x == 0 && a.pg2_out) a.pg2_out[0] = pg0;
    }
    if (a.pg_only) return;

    int steps = 0;
    double tol = a.tol_ptr ? *a.tol_ptr : a.tol_value;
    if (a.ratio > 0.0) tol = a.ratio * sqrt(pg0);
    const int forced = a.forced_ptr ? (int)*a.forced_ptr : a.forced;
    const int kmax = forced >= 0 ? forced : a.inner_max;

    if (L > 0.0) {
        const float invL = (float)(1.0 / L);
        float zp[P], gp[P];
#pragma unroll
        for (int c = 0; c < P; ++c) { zp[c] = z[c]; gp[c] = g[c]; }
        double alpha = 1.0;
        float beta = 0.f;    // weight that produced Y_k from Z_{k-1}, Z_{k-2}
        int k = 1;
        for (; k <= kmax; ++k) {
            // Y_k and grad(Y_k) from the last two iterates.
            float zn[P];
#pragma unroll
            for (int c = 0; c < P; ++c) {
                const float y = fmaf(beta, z[c] - zp[c], z[c]);
                const float gy = fmaf(beta, g[c] - gp[c], g[c]);
                const float v = fmaf(-gy, invL, y);
                zn[c] = (v > 0.f || v != v) ? v : 0.f;
            }
            float gn[P];
            matvec<P>(sW, zn, b, gn);
            const double alpha_n = 0.5 * (1.0 + sqrt(4.0 * alpha * alpha + 1.0));
            beta = (float)((alpha - 1.0) / alpha_n);
            alpha = alpha_n;
#pragma unroll
            for (int c = 0; c < P; ++c) { zp[c] = z[c]; gp[c] = g[c]; z[c] = zn[c]; g[c] = gn[c]; }
            if (forced < 0 && k >= a.inner_min) {
                const double tot = grid_total(active ? pg2_row<P>(z, g) : 0.0, partials, k & 1,
                                              ctl, nblk, ok, s_red, &s_tot);
                if (!ok) break;
                if (!(tot == tot)) {
                    if (blockIdx.x == 0 && threadIdx.x == 0) raise_status(ctl, CNMF_ST_NONFINITE);
                } else if (sqrt(tot) <= tol) {
                    break;
                }
            }
        }
        steps = k > kmax ? kmax : k;
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
        raise_status(ctl, (L != L) ? CNMF_ST_NONFINITE : CNMF_ST_ZERO_LIPS);
    }

    if (active) {
#pragma unroll
        for (int c = 0; c < P; ++c) {
            zrow[c * a.z_cs] = z[c];
            if (a.hist) a.hist[r * a.z_rs + c * a.z_cs] = z[c];
        }
    }
    if (threadIdx.x == 0) {
        if (blockIdx.x == 0) {
            if (a.steps_out) a.steps_out[0] = steps;
            if (a.L_out) a.L_out[0] = L;
            if (a.tol_out) a.tol_out[0] = tol;
            if (a.tol_state && steps >= 1 && steps <= a.inner_min)
                a.tol_state[0] = tol / 10.0;
        }
        if (a.tick_out) {
            __threadfence();
            atomicMax(a.tick_out, (unsigned long long)wall_clock64());
        }
    }
}

template <int P>
hipError_t launch_p(const Dev& d, const KArgs& k, unsigned nblk, double* partials,
                    Control* ctl) {
    hipLaunchKernelGGL(k_nnls<P>, dim3(nblk), dim3(kThreads), 0, d.stream, k, partials, ctl);
    return hipGetLastError();
}

typedef hipError_t (*LaunchFn)(const Dev&, const KArgs&, unsigned, double*, Control*);

template <int... Ps>
struct Table {
    static constexpr LaunchFn fns[sizeof...(Ps)] = {&launch_p<Ps>...};
};
template <int... Ps>
constexpr LaunchFn Table<Ps...>::fns[sizeof...(Ps)];

using PTable = Table<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21,
                     22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32>;

}  // namespace

size_t nnls_partial_doubles(const Dev& d, int64_t rows) {
    (void)rows;
    return 2 * (size_t)d.num_cus;
}

hipError_t nnls(const Dev& d, const NnlsArgs& a, double* partials, Control* ctl) {
    if (a.p < 1 || a.p > 32) return hipErrorInvalidValue;
    const int64_t nblk64 = (a.rows + kThreads - 1) / kThreads;
    if (nblk64 > d.num_cus) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)(nblk64 < 1 ? 1 : nblk64);
    KArgs k;
    k.rows = a.rows;
    k.Z = a.Z;
    k.z_rs = a.z_rs;
    k.z_cs = a.z_cs;
    k.W = a.W;
    k.B = a.B;
    k.L = a.L;
    k.tol_ptr = a.tol_ptr;
    k.tol_value = a.tol_value;
    k.ratio = a.ratio;
    k.tol_state = a.tol_state;
    k.inner_max = a.inner_max;
    k.inner_min = a.inner_min;
    k.forced = a.forced;
    k.forced_ptr = a.forced_ptr;
    k.steps_out = a.steps_out;
    k.L_out = a.L_out;
    k.tol_out = a.tol_out;
    k.pg2_out = a.pg2_out;
    k.hist = a.hist;
    k.tick_out = a.tick_out;
    k.pg_only = a.pg_only ? 1 : 0;
    return PTable::fns[a.p - 1](d, k, nblk, partials, ctl);
}

}  // namespace cnmf
