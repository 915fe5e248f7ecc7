// Batched form: randomized subspace iteration (Sec. 3, Algorithm 2) and the
// compressed NeNMF outer loop (Sec. 3, Algorithm 1) for many independent
// instances.  Every subproblem phase of all instances is one persistent
// launch of k_phase_batched over a schedule of rounds; the outer loop is
// captured in a HIP graph and replayed.
#include <vector>

#include "ctx.hpp"

namespace {

constexpr uint32_t kIdle = 0xffffffffu;

struct Sched {
    std::vector<uint32_t> cells;   // [rounds][slots]
    int rounds = 0;
};

// Workgroups of an instance side with `rows` rows at 64 * tiles rows each.
unsigned blocks_for(int64_t rows, int tiles) {
    const int64_t nb = (rows + 64 * tiles - 1) / (64 * tiles);
    return (unsigned)(nb < 1 ? 1 : nb);
}

// First-fit decreasing: instances (largest first) take contiguous slots of
// the first round with room; a round holds at most `slots` workgroups.
bool pack(const std::vector<unsigned>& nb, int slots, Sched* out) {
    std::vector<int> order(nb.size());
    for (size_t i = 0; i < nb.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nb[a] > nb[b]; });
    std::vector<int> used;
    out->cells.clear();
    for (int i : order) {
        if (nb[i] > (unsigned)slots || nb[i] > 256u) return false;
        int r = 0;
        while (r < (int)used.size() && used[r] + (int)nb[i] > slots) ++r;
        if (r == (int)used.size()) {
            used.push_back(0);
            out->cells.resize(used.size() * slots, kIdle);
        }
        for (unsigned k = 0; k < nb[i]; ++k)
            out->cells[(size_t)r * slots + used[r] + k] = ((uint32_t)i << 12) | k;
        used[r] += (int)nb[i];
    }
    out->rounds = (int)used.size();
    return true;
}

}  // namespace

struct cnmf_batch {
    cnmf_ctx* c = nullptr;
    cnmf_params prm{};
    std::vector<cnmf_instance> inst;
    int tg = 1, tf = 1;
    int slots = 0;
    hipStream_t cap = nullptr;          // capture stream (graphs are launched on the ctx stream)
    // device memory of the batch
    char* mem = nullptr;
    std::vector<uint64_t*> xw;          // per instance: exchange words (kSlotWords)
    std::vector<float*> pG, pF;         // per instance: partial products
    std::vector<double*> st;            // per instance: tol[2], pg2[2]
    std::vector<float*> Gs, Fs;         // per instance: scratch factors for tuning
    unsigned* epoch = nullptr;
    unsigned* done = nullptr;
    // schedules and launch arguments
    uint32_t* schedG = nullptr;
    uint32_t* schedF = nullptr;
    int roundsG = 0, roundsF = 0;
    PhaseArgs* args = nullptr;          // (3 + 2T) blocks of `count`
    size_t args_blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int count_of(const cnmf_batch* b) { return (int)b->inst.size(); }

std::vector<unsigned> side_blocks(const cnmf_batch* b, bool g_side, int tiles) {
    std::vector<unsigned> nb;
    for (const auto& in : b->inst) nb.push_back(blocks_for(g_side ? in.n : in.m, tiles));
    return nb;
}

void free_plan(cnmf_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (b->schedG) (void)hipFree(b->schedG);
    if (b->schedF) (void)hipFree(b->schedF);
    if (b->args) (void)hipFree(b->args);
    b->schedG = b->schedF = nullptr;
    b->args = nullptr;
}

// Per-instance base arguments of the G (rows of G) and F (columns of F)
// subproblems, compressed form (Algorithm 1).
void base_args(const cnmf_batch* b, int i, int tg, int tf, PhaseArgs* ga, PhaseArgs* fa,
               float* G, float* F) {
    const cnmf_instance& in = b->inst[i];
    const int l = in.p + in.nu;
    PhaseArgs base{};
    base.p = in.p;
    base.ell = l;
    base.mode = 2;
    base.slot_s = b->xw[i];
    base.slot_pg = b->xw[i] + 1024;
    base.ctl = b->c->ctl;
    base.inner_max = b->prm.inner_max;
    base.inner_min = b->prm.inner_min;
    base.forced = -1;
    base.dlag = b->c->dlag;
    const unsigned nbG = blocks_for(in.n, tg), nbF = blocks_for(in.m, tf);
    *ga = base;
    ga->rows = in.n;
    ga->Z = G;
    ga->z_rs = in.p;
    ga->z_cs = 1;
    ga->wt = 0;
    ga->D = in.X_R;
    ga->d_rs = l;
    ga->d_cs = 1;
    ga->Q = in.Q_L;
    ga->part_in = b->pF[i];
    ga->nin = (int)nbF;
    ga->part_out = b->pG[i];
    ga->nblk = nbG;
    *fa = base;
    fa->rows = in.m;
    fa->Z = F;
    fa->z_rs = 1;
    fa->z_cs = in.m;
    fa->wt = 1;
    fa->D = in.X_L;
    fa->d_rs = 1;
    fa->d_cs = in.m;
    fa->Q = in.Q_R;
    fa->part_in = b->pG[i];
    fa->nin = (int)nbG;
    fa->part_out = b->pF[i];
    fa->nblk = nbF;
}

// Argument blocks of a solve: 0 F preparation, 1 / 2 initial projected
// gradients (global rule), then G(t), F(t).  forced >= 0 replaces the
// stopping test (tuning runs); scratch selects the tuning copies of G, F.
std::vector<PhaseArgs> solve_args(const cnmf_batch* b, int tg, int tf, int T, int forced,
                                  bool scratch) {
    const int n = count_of(b);
    const bool global = b->prm.stop_rule == CNMF_STOP_GLOBAL;
    std::vector<PhaseArgs> v((size_t)(3 + 2 * T) * n);
    for (int i = 0; i < n; ++i) {
        const cnmf_instance& in = b->inst[i];
        PhaseArgs ga, fa;
        base_args(b, i, tg, tf, &ga, &fa, scratch ? b->Gs[i] : in.G, scratch ? b->Fs[i] : in.F);
        double* st = b->st[i];
        PhaseArgs a = fa;
        a.kind = 2;
        v[(size_t)0 * n + i] = a;
        a = ga;
        a.kind = 1;
        a.pg2_out = st + 2;
        v[(size_t)1 * n + i] = a;
        a = fa;
        a.kind = 1;
        a.pg2_out = st + 3;
        a.tol_init_from = st + 2;
        a.tol_init_out = st;
        a.ratio = b->prm.inner_ratio;
        v[(size_t)2 * n + i] = a;
        for (int t = 0; t < T; ++t) {
            for (int side = 0; side < 2; ++side) {
                a = side == 0 ? ga : fa;
                if (global) {
                    a.tol_ptr = st + side;
                    a.tol_state = st + side;
                } else {
                    a.ratio = b->prm.inner_ratio;
                }
                if (forced >= 0) a.forced = forced;
                else if (in.replay) a.forced_ptr = in.replay + 2 * t + side;
                if (in.steps && !scratch) a.steps_out = in.steps + 2 * t + side;
                v[(size_t)(3 + 2 * t + side) * n + i] = a;
            }
        }
    }
    return v;
}

int build_plan(cnmf_batch* b, int tg, int tf) {
    Sched sg, sf;
    if (!pack(side_blocks(b, true, tg), b->slots, &sg)) return CNMF_EINVAL;
    if (!pack(side_blocks(b, false, tf), b->slots, &sf)) return CNMF_EINVAL;
    free_plan(b);
    const std::vector<PhaseArgs> v = solve_args(b, tg, tf, b->prm.outer_iters, -1, false);
    if (hipMalloc((void**)&b->schedG, sg.cells.size() * 4) != hipSuccess ||
        hipMalloc((void**)&b->schedF, sf.cells.size() * 4) != hipSuccess ||
        hipMalloc((void**)&b->args, v.size() * sizeof(PhaseArgs)) != hipSuccess) {
        free_plan(b);
        return CNMF_ENOMEM;
    }
    if (hipMemcpy(b->schedG, sg.cells.data(), sg.cells.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->schedF, sf.cells.data(), sf.cells.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->args, v.data(), v.size() * sizeof(PhaseArgs), hipMemcpyHostToDevice) != hipSuccess)
        return CNMF_EHIP;
    b->roundsG = sg.rounds;
    b->roundsF = sf.rounds;
    b->args_blocks = v.size() / b->inst.size();
    b->tg = tg;
    b->tf = tf;
    return CNMF_OK;
}

hipError_t launch(const cnmf_batch* b, const Dev& d, const PhaseArgs* block, bool g_side,
                  const uint32_t* schedG, const uint32_t* schedF, int rG, int rF, int tg, int tf) {
    BatchLaunch L;
    L.args = block;
    L.sched = g_side ? schedG : schedF;
    L.count = count_of(b);
    L.rounds = g_side ? rG : rF;
    L.slots = b->slots;
    L.epoch = b->epoch;
    L.done = b->done;
    return phase_batched(d, L, g_side ? tg : tf, b->c->dlag);
}

// Enqueue a whole solve (or a tuning run) whose argument blocks start at args.
hipError_t enqueue(const cnmf_batch* b, const Dev& d, const PhaseArgs* args, int T,
                   const uint32_t* schedG, const uint32_t* schedF, int rG, int rF, int tg,
                   int tf, bool with_pg) {
    const size_t n = b->inst.size();
    hipError_t e = launch(b, d, args, false, schedG, schedF, rG, rF, tg, tf);
    if (e != hipSuccess) return e;
    if (with_pg) {
        if ((e = launch(b, d, args + n, true, schedG, schedF, rG, rF, tg, tf)) != hipSuccess) return e;
        if ((e = launch(b, d, args + 2 * n, false, schedG, schedF, rG, rF, tg, tf)) != hipSuccess)
            return e;
    }
    for (int t = 0; t < T; ++t) {
        if ((e = launch(b, d, args + (3 + 2 * t) * n, true, schedG, schedF, rG, rF, tg, tf)) !=
            hipSuccess)
            return e;
        if ((e = launch(b, d, args + (4 + 2 * t) * n, false, schedG, schedF, rG, rF, tg, tf)) !=
            hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int cnmf_batch_create(cnmf_ctx* c, const cnmf_instance* inst, int32_t count,
                      const cnmf_params* prm, int32_t tiles_g, int32_t tiles_f,
                      cnmf_batch** out) {
    if (!c || !inst || !out || count < 1 || count >= (1 << 20)) return CNMF_EINVAL;
    *out = nullptr;
    for (int i = 0; i < count; ++i) {
        const cnmf_instance& in = inst[i];
        cnmf_params pi = *prm;
        pi.p = in.p;
        pi.nu = in.nu;
        if (check_params(&pi, in.n, in.m, true)) return CNMF_EINVAL;
        if (!in.Q_L || !in.Q_R || !in.X_L || !in.X_R || !in.G || !in.F) return CNMF_EINVAL;
        if (in.X && (in.ldx < in.m)) return CNMF_EINVAL;
    }
    for (int32_t t : {tiles_g, tiles_f})
        if (t != 0 && t != 1 && t != 2 && t != 4) return CNMF_EINVAL;
    cnmf_batch* b = new (std::nothrow) cnmf_batch;
    if (!b) return CNMF_ENOMEM;
    b->c = c;
    b->prm = *prm;
    b->inst.assign(inst, inst + count);
    b->slots = std::min(c->dev.num_cus, 256);
    if (hipSetDevice(c->dev.device) != hipSuccess) { delete b; return CNMF_EHIP; }
    // device state: exchange words, partial products (sized for one tile per
    // workgroup, the most workgroups), tolerance state, scratch factors
    Arena ar;
    std::vector<size_t> oxw, opg, opf, ost, ogs, ofs;
    for (int i = 0; i < count; ++i) {
        const cnmf_instance& in = inst[i];
        oxw.push_back(ar.take<uint64_t>(kSlotWords));
        opg.push_back(ar.take<float>((size_t)blocks_for(in.n, 1) * 1024));
        opf.push_back(ar.take<float>((size_t)blocks_for(in.m, 1) * 1024));
        ost.push_back(ar.take<double>(4));
        ogs.push_back(ar.take<float>((size_t)in.n * in.p));
        ofs.push_back(ar.take<float>((size_t)in.p * in.m));
    }
    const size_t o_ep = ar.take<unsigned>(2);
    if (hipMalloc((void**)&b->mem, ar.off) != hipSuccess) { delete b; return CNMF_ENOMEM; }
    for (int i = 0; i < count; ++i) {
        b->xw.push_back(reinterpret_cast<uint64_t*>(b->mem + oxw[i]));
        b->pG.push_back(reinterpret_cast<float*>(b->mem + opg[i]));
        b->pF.push_back(reinterpret_cast<float*>(b->mem + opf[i]));
        b->st.push_back(reinterpret_cast<double*>(b->mem + ost[i]));
        b->Gs.push_back(reinterpret_cast<float*>(b->mem + ogs[i]));
        b->Fs.push_back(reinterpret_cast<float*>(b->mem + ofs[i]));
    }
    b->epoch = reinterpret_cast<unsigned*>(b->mem + o_ep);
    b->done = b->epoch + 1;
    const unsigned init[2] = {1u, 0u};
    if (hipMemset(b->mem, 0, ar.off) != hipSuccess ||
        hipMemcpy(b->epoch, init, sizeof(init), hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        cnmf_batch_destroy(b);
        return CNMF_EHIP;
    }
    // default tiles: the smallest that fits every instance
    auto fit = [&](bool g_side, int want) {
        if (want) return want;
        for (int t : {1, 2, 4}) {
            Sched s;
            if (pack(side_blocks(b, g_side, t), b->slots, &s)) return t;
        }
        return 0;
    };
    const int tg = fit(true, tiles_g), tf = fit(false, tiles_f);
    if (!tg || !tf) { cnmf_batch_destroy(b); return CNMF_EINVAL; }
    const int rc = build_plan(b, tg, tf);
    if (rc) { cnmf_batch_destroy(b); return rc; }
    *out = b;
    return CNMF_OK;
}

int cnmf_batch_destroy(cnmf_batch* b) {
    if (!b) return CNMF_OK;
    if (b->c) (void)hipSetDevice(b->c->dev.device);
    if (b->c) (void)hipStreamSynchronize(b->c->dev.stream);
    free_plan(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->mem) (void)hipFree(b->mem);
    delete b;
    return CNMF_OK;
}

int cnmf_batch_rsi(cnmf_batch* b) {
    if (!b) return CNMF_EINVAL;
    for (const cnmf_instance& in : b->inst) {
        if (!in.X || !in.omega_L || !in.omega_R) return CNMF_EINVAL;
        cnmf_params pi = b->prm;
        pi.p = in.p;
        pi.nu = in.nu;
        const int rc = rsi_run(b->c, in.n, in.m, in.X, nullptr, in.ldx, &pi, in.omega_L,
                               in.omega_R, in.Q_L, in.Q_R, in.X_L, in.X_R);
        if (rc) return rc;
    }
    return CNMF_OK;
}

int cnmf_batch_tune(cnmf_batch* b, int32_t tune_iters, int32_t* tiles_out) {
    if (!b || tune_iters < 1 || tune_iters > 1000) return CNMF_EINVAL;
    cnmf_ctx* c = b->c;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    const Dev& d = c->dev;
    const int n = count_of(b);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return CNMF_EHIP;
    float best = 3.0e38f;
    int bg = b->tg, bf = b->tf;
    int rc = CNMF_OK;
    for (int tg : {1, 2, 4}) {
        for (int tf : {1, 2, 4}) {
            Sched sg, sf;
            if (!pack(side_blocks(b, true, tg), b->slots, &sg) ||
                !pack(side_blocks(b, false, tf), b->slots, &sf))
                continue;
            const std::vector<PhaseArgs> v = solve_args(b, tg, tf, tune_iters, 10, true);
            uint32_t *dg = nullptr, *df = nullptr;
            PhaseArgs* da = nullptr;
            if (hipMalloc((void**)&dg, sg.cells.size() * 4) != hipSuccess ||
                hipMalloc((void**)&df, sf.cells.size() * 4) != hipSuccess ||
                hipMalloc((void**)&da, v.size() * sizeof(PhaseArgs)) != hipSuccess) {
                rc = CNMF_ENOMEM;
            } else if (hipMemcpy(dg, sg.cells.data(), sg.cells.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                       hipMemcpy(df, sf.cells.data(), sf.cells.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                       hipMemcpy(da, v.data(), v.size() * sizeof(PhaseArgs), hipMemcpyHostToDevice) != hipSuccess) {
                rc = CNMF_EHIP;
            } else {
                float ms = 0.f;
                for (int rep = 0; rep < 2 && rc == CNMF_OK; ++rep) {
                    for (int i = 0; i < n && rc == CNMF_OK; ++i) {
                        const cnmf_instance& in = b->inst[i];
                        if (hipMemcpyAsync(b->Gs[i], in.G, (size_t)in.n * in.p * 4,
                                           hipMemcpyDeviceToDevice, d.stream) != hipSuccess ||
                            hipMemcpyAsync(b->Fs[i], in.F, (size_t)in.p * in.m * 4,
                                           hipMemcpyDeviceToDevice, d.stream) != hipSuccess)
                            rc = CNMF_EHIP;
                    }
                    if (rc) break;
                    if (hipEventRecord(e0, d.stream) != hipSuccess ||
                        enqueue(b, d, da, tune_iters, dg, df, sg.rounds, sf.rounds, tg, tf, false) != hipSuccess ||
                        hipEventRecord(e1, d.stream) != hipSuccess ||
                        hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                        rc = CNMF_EHIP;
                }
                if (rc == CNMF_OK && ms < best) {
                    best = ms;
                    bg = tg;
                    bf = tf;
                }
            }
            if (dg) (void)hipFree(dg);
            if (df) (void)hipFree(df);
            if (da) (void)hipFree(da);
            if (rc) break;
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = build_plan(b, bg, bf);
    if (rc) return rc;
    if (tiles_out) {
        tiles_out[0] = bg;
        tiles_out[1] = bf;
    }
    return CNMF_OK;
}

int cnmf_batch_solve(cnmf_batch* b, int32_t use_graph) {
    if (!b) return CNMF_EINVAL;
    cnmf_ctx* c = b->c;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    const bool global = b->prm.stop_rule == CNMF_STOP_GLOBAL;
    const int T = b->prm.outer_iters;
    if (!use_graph)
        return from_hip(enqueue(b, c->dev, b->args, T, b->schedG, b->schedF, b->roundsG,
                                b->roundsF, b->tg, b->tf, global));
    if (!b->exec) {
        Dev cap = c->dev;
        cap.stream = b->cap;
        if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return CNMF_EHIP;
        const hipError_t e = enqueue(b, cap, b->args, T, b->schedG, b->schedF, b->roundsG,
                                     b->roundsF, b->tg, b->tf, global);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
        if (e != hipSuccess || e2 != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return CNMF_EHIP;
        }
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            b->exec = nullptr;
            return CNMF_EHIP;
        }
    }
    return from_hip(hipGraphLaunch(b->exec, c->dev.stream));
}

}  // extern "C"
