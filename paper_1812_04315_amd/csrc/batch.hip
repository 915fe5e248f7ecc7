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
    double* eig = nullptr;              // per instance: {L, v} per side and parity, contiguous
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
    // randomized subspace iteration (allocated on first use)
    char* rmem = nullptr;
    SweepDesc* rdesc = nullptr;         // right-sweep descriptors, (1 + 2q) x count
    SweepDesc* ldesc = nullptr;         // left-sweep descriptors, (1 + 2q) x count
    TransDesc* tdesc = nullptr;         // 2 x count
    WorkItem* wr = nullptr;             // right sweep / reduce / left sweep / reduce / transposes
    int64_t nwr = 0, nrr = 0, nwl = 0, nrl = 0, nwt = 0;
    WorkItem *wrr = nullptr, *wl = nullptr, *wrl = nullptr, *wt = nullptr;
    OrthArgs* oargs = nullptr;          // 4q arrays of `count`, one per orthonormalisation launch
    uint32_t* osched_n = nullptr;       // round schedules of n-space and m-space panels
    uint32_t* osched_m = nullptr;
    int orounds_n = 0, orounds_m = 0;
    std::vector<uint64_t*> oxw;         // per instance orthonormalisation exchange words
    std::vector<size_t> oxw_words;
    std::vector<unsigned> onb_n, onb_m; // workgroups per panel
    struct RsiPtrs {
        float *oRt, *Yn, *QL, *Ym, *QRt, *oLT, *QRtT, *QLtT, *pr, *pl;
        int64_t ldt;
    };
    std::vector<RsiPtrs> rp;
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
    base.beta = b->c->beta;
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
                double* eg = b->eig + (size_t)i * 4 * kEigWords;
                a.eig_in = eg + (size_t)(2 * side + ((t + 1) & 1)) * kEigWords;
                a.eig_out = eg + (size_t)(2 * side + (t & 1)) * kEigWords;
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
    // no warm start for the first subproblem of either side
    hipError_t e = fill_u64(d, reinterpret_cast<uint64_t*>(b->eig), (int64_t)n * 4 * kEigWords, 0);
    if (e != hipSuccess) return e;
    e = launch(b, d, args, false, schedG, schedF, rG, rF, tg, tf);
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

// Workgroups per panel of one orthonormalisation launch: one per 256 rows
// (orth_batch_blocks), the panels packed into rounds of `slots`.
std::vector<unsigned> orth_share(const std::vector<int64_t>& rows, int slots) {
    std::vector<unsigned> nb;
    for (int64_t r : rows)
        nb.push_back(std::min<unsigned>(orth_batch_blocks(r), (unsigned)std::max(1, slots)));
    return nb;
}

// Workspace, descriptors, work lists and schedules of the batched RSI.
int rsi_prepare(cnmf_batch* b) {
    if (b->rmem) return CNMF_OK;
    const int n = count_of(b);
    const int q = b->prm.q;
    for (const cnmf_instance& in : b->inst) {
        if (!in.X || !in.omega_L || !in.omega_R) return CNMF_EINVAL;
        if (in.ldx % 4 != 0 || (reinterpret_cast<uintptr_t>(in.X) & 15u)) return CNMF_EINVAL;
    }
    std::vector<int64_t> rn, rm;
    for (const cnmf_instance& in : b->inst) {
        rn.push_back(in.n);
        rm.push_back(in.m);
    }
    b->onb_n = orth_share(rn, b->slots);
    b->onb_m = orth_share(rm, b->slots);
    Sched sn, sm;
    if (!pack(b->onb_n, b->slots, &sn) || !pack(b->onb_m, b->slots, &sm)) return CNMF_EINVAL;
    Arena ar;
    struct Off { size_t oRt, Yn, QL, Ym, QRt, oLT, QRtT, QLtT, pr, pl, ox; int64_t ldt; };
    std::vector<Off> off(n);
    for (int i = 0; i < n; ++i) {
        const cnmf_instance& in = b->inst[i];
        const int l = in.p + in.nu;
        const int64_t ldt = (in.m + 3) / 4 * 4;
        Off& o = off[i];
        o.ldt = ldt;
        o.oRt = ar.take<float>((size_t)in.n * l);
        o.Yn = ar.take<float>((size_t)in.n * l);
        o.QL = ar.take<float>((size_t)in.n * l);
        o.Ym = ar.take<float>((size_t)in.m * l);
        o.QRt = ar.take<float>((size_t)in.m * l);
        o.oLT = ar.take<float>((size_t)l * ldt);
        o.QRtT = ar.take<float>((size_t)l * ldt);
        o.QLtT = ar.take<float>((size_t)l * ldt);
        o.pr = ar.take<float>((size_t)in.n * 32);
        o.pl = ar.take<float>((size_t)in.m * 32);
        const unsigned nb = std::max(b->onb_n[i], b->onb_m[i]);
        b->oxw_words.push_back(orth_batch_exchange_words(nb));
        o.ox = ar.take<uint64_t>(b->oxw_words.back());
    }
    const size_t nsteps = 1 + 2 * (size_t)q;
    const size_t o_rd = ar.take<SweepDesc>(nsteps * n);
    const size_t o_ld = ar.take<SweepDesc>(nsteps * n);
    const size_t o_td = ar.take<TransDesc>(2 * (size_t)n);
    const size_t o_oa = ar.take<OrthArgs>((size_t)4 * q * n);
    // work lists
    std::vector<WorkItem> wr, wrr, wl, wrl, wt;
    std::vector<SweepDesc> rd(nsteps * n), ld(nsteps * n);
    std::vector<TransDesc> td(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const cnmf_instance& in = b->inst[i];
        const int l = in.p + in.nu;
        const int nt = l <= 16 ? 16 : 32;
        for (int t = 0; t < (int)((in.n + 31) / 32); ++t) wr.push_back({i, t});
        for (int t = 0; t < (int)((in.m + 255) / 256); ++t) wl.push_back({i, t});
        for (int t = 0; t < (int)((in.n * nt + 255) / 256); ++t) wrr.push_back({i, t});
        for (int t = 0; t < (int)((in.m * nt + 255) / 256); ++t) wrl.push_back({i, t});
        // transposes: Omega_R (l x n) -> n x l, Omega_L (m x l) -> l x ldt
        const int64_t t0 = ((l + 31) / 32) * ((in.n + 31) / 32);
        const int64_t t1 = ((in.m + 31) / 32) * ((l + 31) / 32);
        for (int64_t t = 0; t < t0; ++t) wt.push_back({2 * i, (int)t});
        for (int64_t t = 0; t < t1; ++t) wt.push_back({2 * i + 1, (int)t});
    }
    const size_t o_wr = ar.take<WorkItem>(wr.size());
    const size_t o_wrr = ar.take<WorkItem>(wrr.size());
    const size_t o_wl = ar.take<WorkItem>(wl.size());
    const size_t o_wrl = ar.take<WorkItem>(wrl.size());
    const size_t o_wt = ar.take<WorkItem>(wt.size());
    const size_t o_sn = ar.take<uint32_t>(sn.cells.size());
    const size_t o_sm = ar.take<uint32_t>(sm.cells.size());
    if (hipMalloc((void**)&b->rmem, ar.off) != hipSuccess) {
        b->rmem = nullptr;
        return CNMF_ENOMEM;
    }
    char* base = b->rmem;
    auto F = [&](size_t o) { return reinterpret_cast<float*>(base + o); };
    for (int i = 0; i < n; ++i) {
        const Off& o = off[i];
        cnmf_batch::RsiPtrs r{F(o.oRt), F(o.Yn), F(o.QL), F(o.Ym), F(o.QRt), F(o.oLT),
                              F(o.QRtT), F(o.QLtT), F(o.pr), F(o.pl), o.ldt};
        b->rp.push_back(r);
        b->oxw.push_back(reinterpret_cast<uint64_t*>(base + o.ox));
    }
    for (int i = 0; i < n; ++i) {
        const cnmf_instance& in = b->inst[i];
        const cnmf_batch::RsiPtrs& r = b->rp[i];
        const int l = in.p + in.nu;
        td[2 * i] = TransDesc{l, in.n, in.omega_R, in.n, r.oRt, l};
        td[2 * i + 1] = TransDesc{in.m, l, in.omega_L, l, r.oLT, r.ldt};
        // right sweeps: step 0 X oL, then per k: X Q_R^(k-1)^T... (as rsi_run)
        size_t sr = 0, sl = 0;
        auto R_ = [&](const float* AT, float* Y) {
            sweep_desc_right(&rd[sr++ * n + i], in.n, in.m, in.X, in.ldx, l, AT, r.ldt, r.pr, Y, l);
        };
        auto L_ = [&](const float* B, float* Z, bool trans) {
            sweep_desc_left(&ld[sl++ * n + i], in.n, in.m, in.X, in.ldx, l, B, l, r.pl, Z,
                            trans ? in.m : l, trans);
        };
        R_(r.oLT, r.Yn);
        L_(r.oRt, r.Ym, false);
        for (int k = 1; k <= q; ++k) {
            L_(r.QL, r.Ym, false);
            R_(r.QRtT, r.Yn);
            R_(r.QLtT, in.X_R);
            if (k < q) L_(in.Q_L, r.Ym, false);
            else L_(in.Q_L, in.X_L, true);
        }
    }
    b->rdesc = reinterpret_cast<SweepDesc*>(base + o_rd);
    b->ldesc = reinterpret_cast<SweepDesc*>(base + o_ld);
    b->tdesc = reinterpret_cast<TransDesc*>(base + o_td);
    b->oargs = reinterpret_cast<OrthArgs*>(base + o_oa);
    b->wr = reinterpret_cast<WorkItem*>(base + o_wr);
    b->wrr = reinterpret_cast<WorkItem*>(base + o_wrr);
    b->wl = reinterpret_cast<WorkItem*>(base + o_wl);
    b->wrl = reinterpret_cast<WorkItem*>(base + o_wrl);
    b->wt = reinterpret_cast<WorkItem*>(base + o_wt);
    b->osched_n = reinterpret_cast<uint32_t*>(base + o_sn);
    b->osched_m = reinterpret_cast<uint32_t*>(base + o_sm);
    b->nwr = (int64_t)wr.size();
    b->nrr = (int64_t)wrr.size();
    b->nwl = (int64_t)wl.size();
    b->nrl = (int64_t)wrl.size();
    b->nwt = (int64_t)wt.size();
    b->orounds_n = sn.rounds;
    b->orounds_m = sm.rounds;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return bytes == 0 || hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(b->rdesc, rd.data(), rd.size() * sizeof(SweepDesc)) ||
        !up(b->ldesc, ld.data(), ld.size() * sizeof(SweepDesc)) ||
        !up(b->tdesc, td.data(), td.size() * sizeof(TransDesc)) ||
        !up(b->wr, wr.data(), wr.size() * sizeof(WorkItem)) ||
        !up(b->wrr, wrr.data(), wrr.size() * sizeof(WorkItem)) ||
        !up(b->wl, wl.data(), wl.size() * sizeof(WorkItem)) ||
        !up(b->wrl, wrl.data(), wrl.size() * sizeof(WorkItem)) ||
        !up(b->wt, wt.data(), wt.size() * sizeof(WorkItem)) ||
        !up(b->osched_n, sn.cells.data(), sn.cells.size() * 4) ||
        !up(b->osched_m, sm.cells.data(), sm.cells.size() * 4))
        return CNMF_EHIP;
    for (int i = 0; i < n; ++i)
        if (fill_u64(b->c->dev, b->oxw[i], (int64_t)b->oxw_words[i], 0) != hipSuccess)
            return CNMF_EHIP;
    return CNMF_OK;
}

}  // namespace

extern "C" {

int cnmf_batch_create(cnmf_ctx* c, const cnmf_instance* inst, int32_t count,
                      const cnmf_params* prm, int32_t tiles_g, int32_t tiles_f,
                      cnmf_batch** out) {
    if (!c || !inst || !out || count < 1 || count >= (1 << 20)) return CNMF_EINVAL;
    *out = nullptr;
    // the batched form runs the Nesterov inner loop without restart and
    // without a time budget
    if (!prm || prm->solver != CNMF_SOLVER_NESTEROV || prm->restart != CNMF_RESTART_NONE ||
        prm->time_budget != 0.0)
        return CNMF_EINVAL;
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
    const size_t o_eig = ar.take<double>((size_t)count * 4 * kEigWords);
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
    b->eig = reinterpret_cast<double*>(b->mem + o_eig);
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
    if (b->rmem) (void)hipFree(b->rmem);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->mem) (void)hipFree(b->mem);
    delete b;
    return CNMF_OK;
}

int cnmf_batch_rsi(cnmf_batch* b) {
    if (!b) return CNMF_EINVAL;
    cnmf_ctx* c = b->c;
    if (hipSetDevice(c->dev.device) != hipSuccess) return CNMF_EHIP;
    const int rc = rsi_prepare(b);
    if (rc) return rc;
    const Dev& d = c->dev;
    const int n = count_of(b);
    const int q = b->prm.q;
    // fresh tags for the 2 + 3q - 1 orthonormalisation launches
    const int north = 4 * q;
    std::vector<OrthArgs> oa((size_t)north * n);
    std::vector<unsigned> seqs(north);
    bool wrapped = false;
    for (int j = 0; j < north; ++j) {
        const unsigned before = c->seq;
        if (next_seq(c, &seqs[j]) != hipSuccess) return CNMF_EHIP;
        if (seqs[j] < before) wrapped = true;
    }
    if (wrapped)
        for (int i = 0; i < n; ++i)
            CK(fill_u64(d, b->oxw[i], (int64_t)b->oxw_words[i], 0));
    // orth launch j: panels of every instance (n-space or m-space)
    auto set_orth = [&](int j, int i, bool nspace, const float* Y, float* Q, float* QT) {
        const cnmf_instance& in = b->inst[i];
        const cnmf_batch::RsiPtrs& r = b->rp[i];
        const int l = in.p + in.nu;
        oa[(size_t)j * n + i] =
            nspace ? orth_args(in.n, l, Y, r.oRt, false, b->prm.tau2, Q, nullptr, 0, nullptr,
                               b->oxw[i], seqs[j], c->ctl, b->onb_n[i])
                   : orth_args(in.m, l, Y, in.omega_L, false, b->prm.tau2, Q, QT, r.ldt,
                               nullptr, b->oxw[i], seqs[j], c->ctl, b->onb_m[i]);
    };
    // the orthonormalisation sequence of Algorithm 2 (see rsi_run)
    int j = 0;
    std::vector<std::pair<int, bool>> order;   // (launch, n-space)
    for (int i = 0; i < n; ++i) {
        const cnmf_instance& in = b->inst[i];
        const cnmf_batch::RsiPtrs& r = b->rp[i];
        int jj = 0;
        set_orth(jj++, i, true, r.Yn, r.QL, nullptr);
        set_orth(jj++, i, false, r.Ym, r.QRt, r.QRtT);
        for (int k = 1; k <= q; ++k) {
            set_orth(jj++, i, false, r.Ym, in.Q_R, r.QLtT);
            set_orth(jj++, i, true, r.Yn, in.Q_L, nullptr);
            if (k < q) {
                set_orth(jj++, i, true, in.X_R, r.QL, nullptr);
                set_orth(jj++, i, false, r.Ym, r.QRt, r.QRtT);
            }
        }
        j = jj;
    }
    const int used = j;
    CK(hipMemcpyAsync(b->oargs, oa.data(), (size_t)used * n * sizeof(OrthArgs),
                      hipMemcpyHostToDevice, d.stream));
    CK(hipStreamSynchronize(d.stream));   // oa is pageable host memory
    auto orth_launch = [&](int jl, bool nspace) -> hipError_t {
        return orth_batched(d, b->oargs + (size_t)jl * n, nspace ? b->osched_n : b->osched_m,
                            nspace ? b->orounds_n : b->orounds_m, b->slots);
    };
    auto right = [&](int step) -> hipError_t {
        const SweepDesc* s = b->rdesc + (size_t)step * n;
        hipError_t e = sweep_right_batched(d, s, b->wr, b->nwr);
        if (e != hipSuccess) return e;
        return reduce_batched(d, s, b->wrr, b->nrr, false);
    };
    auto left = [&](int step) -> hipError_t {
        const SweepDesc* s = b->ldesc + (size_t)step * n;
        hipError_t e = sweep_left_batched(d, s, b->wl, b->nwl);
        if (e != hipSuccess) return e;
        return reduce_batched(d, s, b->wrl, b->nrl, true);
    };
    CK(transpose_batched(d, b->tdesc, b->wt, b->nwt));
    int jo = 0, sr = 0, sl = 0;
    CK(right(sr++));
    CK(orth_launch(jo++, true));
    CK(left(sl++));
    CK(orth_launch(jo++, false));
    for (int k = 1; k <= q; ++k) {
        CK(left(sl++));
        CK(orth_launch(jo++, false));
        CK(right(sr++));
        CK(orth_launch(jo++, true));
        CK(right(sr++));
        CK(left(sl++));
        if (k < q) {
            CK(orth_launch(jo++, true));
            CK(orth_launch(jo++, false));
        }
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
