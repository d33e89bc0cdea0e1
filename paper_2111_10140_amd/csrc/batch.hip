// Batched products: every (problem, window, right-hand side) of a set of
// products runs in one launch per stage and kernel signature.
//
// build() lays out one WinInst per instance (window data of the plan, the
// input column, and a private slice of one work-space allocation: grid,
// spread regions, per-tile region sums, interpolated values); a prediction
// takes two per window and column, one that spreads the training points and
// convolves, and one that gathers at the targets from the same grid (the
// two node sets of the fast sum, Sec. 4.2).  It groups the
// instances of each stage by kernel signature, and uploads the instance and
// group tables.  run() issues the stages in order: permute, spread, tile
// sum, fold, convolve (one pass per axis), gather, combine.  Nothing is allocated or
// copied in run(), so it can be captured in a hipGraph.
#include <algorithm>
#include <map>
#include <tuple>

#include "anova_internal.h"

namespace anova {

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Sizes {
    size_t grid, priv, treg, tmp;
};

Sizes instance_sizes(const WindowPlan &w, size_t es, bool own_grid) {
    Sizes z{};
    z.grid = own_grid ? align256(w.grid_elems() * es) : 0;
    z.priv = align256((size_t)w.n_regions * w.region_elems() * es);
    z.treg = w.n_regions != w.n_nonempty ? align256((size_t)w.n_nonempty * w.region_elems() * es) : 0;
    z.tmp = align256((size_t)w.n_points * es);
    return z;
}

// Instance fields taken from a window's plan.
void fill_inst(WinInst &wi, const WindowPlan &w, const double *alpha, void *grid) {
    wi.nodes = w.nodes.ptr;
    wi.perm = w.perm.as<int32_t>();
    wi.subs = w.subs.as<SubProblem>();
    wi.tiles_ne = w.tiles_ne.as<int32_t>();
    wi.cell_start = w.cell_start.as<int32_t>();
    wi.src_sub = w.src_sub.as<int32_t>();
    wi.fold_pairs = w.fold_pairs.as<int2>();
    wi.fold_start = w.fold_start.as<int32_t>();
    wi.fold_tiles = w.fold_tiles.as<int32_t>();
    wi.fold_act = w.fold_act;
    wi.fold_len = w.fold_len;
    wi.poly = w.poly.ptr;
    wi.bconv = w.bconv.ptr;
    wi.ctaps = w.ctaps.ptr;
    wi.twiddle = w.twiddle.ptr;
    wi.alpha = alpha;
    wi.grid = grid;
    wi.n = w.n;
    wi.tile = w.tile;
    wi.tpd = w.tiles_per_dim;
    wi.vol = (int32_t)w.region_elems();
    wi.n_sub = (int32_t)w.n_sub;
    wi.n_nonempty = (int32_t)w.n_nonempty;
    wi.n_tiles = (int32_t)w.n_tiles;
    wi.n_regions = (int32_t)w.n_regions;
    wi.N = (int32_t)w.n_points;
    wi.dA = w.dA;
    wi.width = 2 * w.m;
    wi.chunks = w.dense ? w.chunks : 0;
}

}  // namespace

size_t problem_work_bytes(const BatchProblem &bp) {
    const size_t es = problem_precision(bp) == ANOVA_FP64 ? 8 : 4;
    const std::vector<WindowPlan> &wins = problem_windows(bp);
    size_t total = 0;
    for (int c = 0; c < bp.nrhs; ++c)
        for (int l = 0; l < bp.plan->P; ++l) {
            if (bp.only_window >= 0 && l != bp.only_window) continue;
            const Sizes z = instance_sizes(wins[l], es, bp.grid_override == nullptr);
            total += z.grid + z.priv + z.treg + z.tmp;
            if (bp.predict) total += align256((size_t)bp.plan->tgt[l].n_points * es);
        }
    return total;
}

size_t Batch::device_bytes() const {
    return d_insts.bytes + d_combs.bytes + d_cwins.bytes + d_tables.bytes + work.bytes;
}

bool Batch::same(const std::vector<BatchProblem> &problems) const {
    if (problems.size() != probs.size()) return false;
    for (size_t i = 0; i < problems.size(); ++i) {
        const BatchProblem &a = problems[i], &b = probs[i];
        if (a.plan != b.plan || a.alpha != b.alpha || a.out != b.out || a.nrhs != b.nrhs ||
            a.ld != b.ld || a.ld_out != b.ld_out || a.beta != b.beta ||
            a.only_window != b.only_window ||
            a.grid_override != b.grid_override || a.work != b.work ||
            a.residual != b.residual || a.predict != b.predict || a.hooks || b.hooks)
            return false;
    }
    return true;
}

void Batch::build(const std::vector<BatchProblem> &problems, const ExternalSpace *ext) {
    ANOVA_REQUIRE(!problems.empty(), "empty batch");
    precision = problem_precision(problems[0]);
    for (const BatchProblem &bp : problems) {
        ANOVA_REQUIRE(problem_precision(bp) == precision,
                      "a batch mixes float32 and float64 products");
        ANOVA_REQUIRE(!bp.predict || ((int)bp.plan->tgt.size() == bp.plan->P &&
                                      bp.only_window < 0 && !bp.grid_override && !bp.residual),
                      "prediction needs a plan with targets, all windows and its own grids");
    }
    const size_t es = precision == ANOVA_FP64 ? 8 : 4;
    insts.clear();
    roles.clear();
    combs.clear();
    cwins.clear();
    groups.clear();
    // ---- instances and work-space layout
    struct Slot {
        size_t grid, priv, treg, tmp;
    };
    std::vector<Slot> slots;
    std::vector<char *> slot_base;  // nullptr: the batch's own work space
    std::vector<int64_t> grid_of;   // -1, or the instance whose grid this one gathers from
    std::vector<int64_t> cwin_inst; // instance whose values each combine window reads
    size_t total = 0;
    for (const BatchProblem &bp : problems) {
        anova_plan_s *p = bp.plan;
        size_t own = 0;  // offsets inside the caller's work space
        size_t &off = bp.work ? own : total;
        for (int c = 0; c < bp.nrhs; ++c) {
            CombInst ci{};
            const int64_t ldo = bp.ld_out >= 0 ? bp.ld_out : bp.ld;
            ci.out = bp.out ? bp.out + (size_t)c * ldo : nullptr;
            // a prediction has no shift (its output rows are other points)
            ci.alpha = bp.predict ? nullptr : bp.alpha + (size_t)c * bp.ld;
            ci.beta = bp.predict ? 0.0 : bp.beta;
            ci.N = (int32_t)(bp.predict ? p->Nz : p->N);
            ci.win0 = (int32_t)cwins.size();
            ci.accumulate = bp.only_window >= 0 ? 1 : 0;
            if (bp.hooks) ci.hook = bp.hooks[c];
            int nw = 0;
            for (int l = 0; l < p->P; ++l) {
                if (bp.only_window >= 0 && l != bp.only_window) continue;
                const WindowPlan &w = problem_windows(bp)[l];
                const Sizes z = instance_sizes(w, es, bp.grid_override == nullptr);
                Slot sl{off, off + z.grid, off + z.grid + z.priv, off + z.grid + z.priv + z.treg};
                off += z.grid + z.priv + z.treg + z.tmp;
                slots.push_back(sl);
                slot_base.push_back(static_cast<char *>(bp.work));
                WinInst wi{};
                // the grid is patched below when owned
                fill_inst(wi, w, bp.alpha + (size_t)c * bp.ld, bp.grid_override);
                insts.push_back(wi);
                roles.push_back(bp.predict ? 1 : 3);
                grid_of.push_back(-1);
                if (bp.predict) {
                    // the targets: no grid, regions or sums of their own
                    const WindowPlan &v = p->tgt[l];
                    const size_t tz = align256((size_t)v.n_points * es);
                    slots.push_back(Slot{off, off, off, off});
                    off += tz;
                    slot_base.push_back(static_cast<char *>(bp.work));
                    WinInst wt{};
                    fill_inst(wt, v, nullptr, nullptr);
                    grid_of.push_back((int64_t)insts.size() - 1);
                    insts.push_back(wt);
                    roles.push_back(2);
                }
                cwin_inst.push_back((int64_t)insts.size() - 1);
                cwins.push_back(CombineWin{nullptr, w.eta});
                ++nw;
            }
            ci.P = nw;
            combs.push_back(ci);
        }
    }
    // batch-owned work space: an allocation of the batch's own, or the
    // start of the external space (the tables follow it there)
    char *own_work = nullptr;
    if (ext) {
        work.release();
        own_work = ext->base;
    } else {
        if (total == 0)
            work.release();
        else if (!work.ptr || work.bytes < total)
            work.alloc(total);
        own_work = static_cast<char *>(work.ptr);
    }
    for (size_t i = 0; i < insts.size(); ++i) {
        char *base = slot_base[i] ? slot_base[i] : own_work;
        if (grid_of[i] >= 0)
            insts[i].grid = insts[(size_t)grid_of[i]].grid;  // built before it
        else if (!insts[i].grid)
            insts[i].grid = base + slots[i].grid;
        insts[i].priv = base + slots[i].priv;
        insts[i].treg = base + slots[i].treg;
        insts[i].tmp = base + slots[i].tmp;
    }
    for (size_t k = 0; k < cwins.size(); ++k) cwins[k].tmp = insts[(size_t)cwin_inst[k]].tmp;
    // ---- groups: key -> member list, per stage
    std::vector<int32_t> table;  // all members and prefixes, packed
    struct PendingGroup {
        BatchGroup g;
        std::vector<int32_t> members, blocks;
    };
    std::vector<PendingGroup> pending;
    auto add_stage = [&](int stage, auto key_of, auto blocks_of, auto fill) {
        std::map<std::tuple<int, int, int, int, int, int>, size_t> idx;
        const unsigned role = stage == kStageGather ? 2u : 1u;
        for (size_t i = 0; i < insts.size(); ++i) {
            if (!(roles[i] & role)) continue;
            int b = 0;
            if (!blocks_of(insts[i], b) || b <= 0) continue;
            const auto key = key_of(insts[i]);
            auto it = idx.find(key);
            if (it == idx.end()) {
                PendingGroup pg;
                pg.g.stage = stage;
                fill(pg.g, insts[i]);
                it = idx.emplace(key, pending.size()).first;
                pending.push_back(pg);
            }
            pending[it->second].members.push_back((int32_t)i);
            pending[it->second].blocks.push_back(b);
        }
    };
    // permute: coefficients into each window's sorted order (per-point
    // kernels only: the per-cell spread reads them through the permutation)
    add_stage(
        kStagePermute, [](const WinInst &) { return std::make_tuple(0, 0, 0, 0, 0, 0); },
        [](const WinInst &w, int &b) {
            if (w.cell_start != nullptr) return false;
            b = (w.N + permute_span() - 1) / permute_span();
            return true;
        },
        [](BatchGroup &, const WinInst &) {});
    // spread
    add_stage(
        kStageSpread,
        [](const WinInst &w) {
            return std::make_tuple(w.cell_start != nullptr ? 1 : 0, w.dA, w.width, w.tile, 0, 0);
        },
        [](const WinInst &w, int &b) {
            b = w.cell_start != nullptr ? w.n_regions : w.n_sub;
            return true;
        },
        [](BatchGroup &g, const WinInst &w) {
            g.cell = w.cell_start != nullptr ? 1 : 0;
            g.dA = w.dA;
            g.W = w.width;
            g.tile = w.tile;
        });
    // tile sum (instances whose tiles hold several regions)
    add_stage(
        kStageTileSum, [](const WinInst &) { return std::make_tuple(0, 0, 0, 0, 0, 0); },
        [](const WinInst &w, int &b) {
            if (w.n_regions == w.n_nonempty) return false;
            b = w.n_nonempty * ((w.vol + 255) / 256);
            return true;
        },
        [](BatchGroup &, const WinInst &) {});
    // fold
    add_stage(
        kStageFold, [](const WinInst &w) { return std::make_tuple(w.dA, 0, 0, 0, 0, 0); },
        [](const WinInst &w, int &b) {
            b = fold_blocks(w);
            return true;
        },
        [](BatchGroup &g, const WinInst &w) { g.dA = w.dA; });
    // convolve: per axis by FFT, or (small grids of 2 or 3 dimensions) by
    // direct taps, axes 0 and 1 by planes, then axis 2
    for (int pass = 0; pass < 3; ++pass) {
        add_stage(
            kStageConvolve, [](const WinInst &w) { return std::make_tuple(w.n, w.dA, 0, 0, 0, 0); },
            [pass, es](const WinInst &w, int &b) {
                if (pass >= w.dA) return false;
                if (convolve_direct(w.n, w.dA)) {
                    if (pass == 1) return false;  // done with axis 0
                    b = pass == 0 && w.dA == 2 ? 1 : w.n;  // planes, or columns of one y
                    return true;
                }
                int nlines = 1;
                for (int t = 1; t < w.dA; ++t) nlines *= w.n;
                const int nq = (nlines + 1) / 2;
                const int np = convolve_lines_per_block(w.n, nq, (int)es);
                b = (nq + np - 1) / np;
                return true;
            },
            [pass, es](BatchGroup &g, const WinInst &w) {
                g.n = w.n;
                g.axis = convolve_direct(w.n, w.dA) ? (pass == 0 ? -1 : -2) : pass;
                // instances of one group share n and d_A, hence the line count
                int nlines = 1;
                for (int t = 1; t < w.dA; ++t) nlines *= w.n;
                g.np = convolve_lines_per_block(w.n, (nlines + 1) / 2, (int)es);
            });
    }
    // gather
    add_stage(
        kStageGather,
        [](const WinInst &w) {
            return std::make_tuple(w.cell_start != nullptr ? 1 : 0, w.dA, w.width, w.tile, 0, 0);
        },
        [](const WinInst &w, int &b) {
            b = w.cell_start != nullptr ? w.n_regions : w.n_sub;
            return true;
        },
        [](BatchGroup &g, const WinInst &w) {
            g.cell = w.cell_start != nullptr ? 1 : 0;
            g.dA = w.dA;
            g.W = w.width;
            g.tile = w.tile;
        });
    // pack tables
    std::vector<size_t> moff, poff;
    for (PendingGroup &pg : pending) {
        moff.push_back(table.size());
        table.insert(table.end(), pg.members.begin(), pg.members.end());
        poff.push_back(table.size());
        int acc = 0;
        table.push_back(0);
        for (int b : pg.blocks) {
            acc += b;
            table.push_back(acc);
        }
        pg.g.blocks = acc;
        pg.g.cnt = (int)pg.members.size();
    }
    // combine prefix
    const size_t coff = table.size();
    {
        int acc = 0;
        table.push_back(0);
        for (const CombInst &ci : combs) {
            acc += (ci.N + combine_span() - 1) / combine_span();
            table.push_back(acc);
        }
        comb_blocks = acc;
        comb_cnt = (int)combs.size();
    }
    const int32_t *tb = nullptr;
    if (ext) {
        // layout of the external space: work, tables, instances, combine
        // columns, combine windows (each 256-byte aligned); every size is
        // checked before anything is written
        const size_t o_tab = align256(total);
        const size_t o_ins = o_tab + align256(table.size() * sizeof(int32_t));
        const size_t o_cmb = o_ins + align256(insts.size() * sizeof(WinInst));
        const size_t o_cwn = o_cmb + align256(combs.size() * sizeof(CombInst));
        const size_t end = o_cwn + align256(cwins.size() * sizeof(CombineWin));
        if (end > ext->bytes)
            throw Error{ANOVA_E_INVALID,
                        "the product needs " + std::to_string(end) +
                            " bytes of static work space, above its maximum of " +
                            std::to_string(ext->bytes)};
        auto put = [&](size_t off, const void *src, size_t bytes) {
            if (bytes)
                ANOVA_HIP_CHECK(hipMemcpy(ext->base + off, src, bytes, hipMemcpyHostToDevice));
        };
        put(o_tab, table.data(), table.size() * sizeof(int32_t));
        put(o_ins, insts.data(), insts.size() * sizeof(WinInst));
        put(o_cmb, combs.data(), combs.size() * sizeof(CombInst));
        put(o_cwn, cwins.data(), cwins.size() * sizeof(CombineWin));
        d_tables.release();
        d_insts.release();
        d_combs.release();
        d_cwins.release();
        tb = reinterpret_cast<const int32_t *>(ext->base + o_tab);
        dev_insts = reinterpret_cast<const WinInst *>(ext->base + o_ins);
        dev_combs = reinterpret_cast<const CombInst *>(ext->base + o_cmb);
        dev_cwins = reinterpret_cast<const CombineWin *>(ext->base + o_cwn);
    } else {
        upload(d_tables, table);
        upload(d_insts, insts);
        upload(d_combs, combs);
        upload(d_cwins, cwins);
        tb = d_tables.as<int32_t>();
        dev_insts = d_insts.as<WinInst>();
        dev_combs = d_combs.as<CombInst>();
        dev_cwins = d_cwins.as<CombineWin>();
    }
    for (size_t k = 0; k < pending.size(); ++k) {
        pending[k].g.members = tb + moff[k];
        pending[k].g.prefix = tb + poff[k];
        groups.push_back(pending[k].g);
    }
    comb_prefix = tb + coff;
    probs = problems;
}

Batch::~Batch() {
    if (last_run_) (void)hipEventDestroy(last_run_);
}

void Batch::record_run(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    ANOVA_HIP_CHECK(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) {
        captured_ = true;
        return;
    }
    if (!last_run_) ANOVA_HIP_CHECK(hipEventCreateWithFlags(&last_run_, hipEventDisableTiming));
    ANOVA_HIP_CHECK(hipEventRecord(last_run_, s));
    run_recorded_ = true;
}

void Batch::wait_last_run() {
    if (run_recorded_) ANOVA_HIP_CHECK(hipEventSynchronize(last_run_));
    run_recorded_ = false;
}

void run_cached(std::vector<std::unique_ptr<Batch>> &cache, const std::vector<BatchProblem> &probs,
                hipStream_t s, anova_plan_s *timing) {
    // most recently used last
    size_t k = cache.size();
    for (size_t i = 0; i < cache.size(); ++i)
        if (cache[i]->same(probs)) k = i;
    if (k == cache.size()) {
        size_t victim = cache.size();
        if (cache.size() >= kBatchCache)
            for (size_t i = 0; i < cache.size() && victim == cache.size(); ++i)
                if (!cache[i]->captured()) victim = i;
        if (victim == cache.size()) {
            std::unique_ptr<Batch> b(new Batch());
            b->build(probs);
            cache.push_back(std::move(b));
        } else {
            cache[victim]->wait_last_run();
            cache[victim]->build(probs);
            k = victim;
        }
    }
    if (k < cache.size()) {
        std::unique_ptr<Batch> b = std::move(cache[k]);
        cache.erase(cache.begin() + k);
        cache.push_back(std::move(b));
    }
    cache.back()->run(s, timing);
    cache.back()->record_run(s);
}

void Batch::run(hipStream_t s, anova_plan_s *timing, unsigned mask) const {
    const WinInst *di = dev_insts;
    size_t k = 0;
    // groups are stored stage by stage in execution order
    while (k < groups.size()) {
        const int stage = groups[k].stage;
        size_t e = k;
        while (e < groups.size() && groups[e].stage == stage &&
               (stage != kStageConvolve || groups[e].axis == groups[k].axis))
            ++e;
        if (mask & (1u << stage)) {
            timed_launch(timing, stage, s, [&] {
                for (size_t q = k; q < e; ++q) run_group(groups[q], precision, di, s);
            });
        }
        k = e;
    }
    if ((mask & (1u << kStageCombine)) && comb_cnt > 0) {
        timed_launch(timing, kStageCombine, s, [&] {
            run_combine(dev_combs, dev_cwins, comb_prefix, comb_cnt,
                        comb_blocks, precision, s);
        });
    }
}

}  // namespace anova
