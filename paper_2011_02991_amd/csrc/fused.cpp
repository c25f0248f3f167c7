// fused.cpp -- host executor of the fused metric: forward state, column
// seeds and the tiled sweep passes of every column (see sweep.hpp, api.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "fused.hpp"

#include "gram_kernels.hpp"

namespace qng {

namespace {

#define FCHECK(call)                                                                                  \
    do {                                                                                              \
        hipError_t _e = (call);                                                                       \
        if (_e != hipSuccess) fail(QNG_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

DevMat2 to_dev(const Mat2 &m) {
    return DevMat2{m.a.real(), m.a.imag(), m.b.real(), m.b.imag(), m.c.real(), m.c.imag(), m.d.real(), m.d.imag()};
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// The shears of the fixed rotations of a lowered circuit (rows by gate position).
void fill_fixed_shears(const Circuit &c, const std::vector<Mat2> &adj, std::vector<double> &mats) {
    for (int pos = 0; pos < c.M; ++pos) {
        if (!c.is_fixed_rotation(pos)) continue;
        const int kind = c.gates[pos].kind;
        const Shear sh = adjoint_shear(kind == QNG_RX ? AX_X : kind == QNG_RY ? AX_Y : AX_Z, adj[pos]);
        mats[(size_t)pos * 8 + 0] = sh.u;
        mats[(size_t)pos * 8 + 1] = sh.w;
    }
}

struct Launch {
    uint32_t item_begin = 0, n_items = 0, total_tiles = 0, task_begin = 0, n_tasks = 0;
};
struct Group {
    int col_begin = 0, col_end = 0;
    size_t launch_begin = 0, launch_end = 0;
};

}  // namespace

size_t fused_scratch_bytes(const SweepPlan &plan, const FusedRun &fr, int M) {
    size_t b = 0;
    b += align256((size_t)M * 64 + 64);                                  // matrix table (FP64)
    b += align256((size_t)M * 32 + 64);                                  // matrix table (FP32)
    b += align256((size_t)M * 64 + 64);                                  // forward matrices (FP64)
    b += align256((size_t)(M + 1) * 64 + 64);                            // the same negated, and -I
    b += align256(plan.dev_passes.size() * sizeof(DevPass) + 64);       // passes
    b += align256(plan.dev_ops.size() * sizeof(DevOp) + 64);            // ops
    b += align256(plan.dev_maps.size() * sizeof(DevMap) + 64);          // thread mappings
    b += align256(plan.dev_passes.size() * sizeof(LaunchItem) + 64);    // one item per pass
    b += align256(((size_t)plan.P * plan.P / 2 + plan.P) * sizeof(ReduceTask) + 64);  // elements and seeds
    b += align256((size_t)plan.P + 1 + 64);                              // signs (derivative-state variant)
    if (plan.forward) {
        const SweepPlan &fp = *plan.forward;
        b += align256((size_t)M * 64 + 64);                              // the gates' own shears (FP64)
        b += align256((size_t)M * 32 + 64);                              // (FP32)
        b += align256(fp.dev_passes.size() * sizeof(DevPass) + 64);
        b += align256(fp.dev_ops.size() * sizeof(DevOp) + 64);
        b += align256(fp.dev_maps.size() * sizeof(DevMap) + 64);
        b += align256(fp.dev_passes.size() * sizeof(LaunchItem) + 64);
    }
    b += align256(fr.partial_elems * 16);
    return b;
}

template <typename R>
int run_fused_metric(const SweepPlan &plan, const FusedRun &fr, const Circuit &c, const std::vector<Mat2> &fwd,
                     const std::vector<Mat2> &adj, const FusedBuffers &buf, hipStream_t st, qng_stats *stats,
                     bool profile, int reg_mode, bool real_products) {
    const int n = c.n;
    const size_t V = buf.state_bytes;
    const uint32_t tiles = 1u << (n - plan.m);
    const int ncols = (int)plan.cols.size();   // column blocks
    const int B = fr.B;                        // blocks swept concurrently
    const int W = plan.width;                  // phi registers per block
    if (W > 1 && buf.traw != buf.lraw + 2 * (size_t)c.P * c.P)
        fail(QNG_E_DEVICE, "fused sweep: T must follow L in memory for column blocks (internal)");
    auto state = [&](int k) -> void * { return buf.states + (size_t)k * V; };
    const bool states = buf.xi != nullptr;   // derivative-state variant
    // block b of a group: lambda, then phi registers 0 .. W-1 (the top column's is W-1)
    auto reg = [&](int b, int k) -> void * { return state(1 + (W + 1) * b + k); };
    // the phi register k of the block whose top column is s: the kept state of
    // its column in the derivative-state variant (the lowest block's register
    // below column 1 is never seeded and goes to the dummy state)
    char *const xi_chunk = buf.xi_chunk ? buf.xi_chunk : buf.xi + 2 * V;
    auto xi_of = [&](int s, int b, int k) -> void * {
        if (!states) return reg(b, 1 + k);
        const int col = s - (W - 1) + k;
        return col >= 1 ? (void *)(xi_chunk + (size_t)(col - buf.chunk_col0) * V) : (void *)buf.dummy;
    };
    const int blk_begin = buf.blk_begin, blk_end = buf.blk_end < 0 ? ncols : std::min(buf.blk_end, ncols);

    // ---- launch schedule (host)
    std::vector<LaunchItem> items;
    std::vector<ReduceTask> tasks;
    std::vector<Launch> launches;
    std::vector<Group> groups;
    int64_t elements = 0;
    items.reserve(plan.dev_passes.size());
    for (int g0 = blk_begin; g0 < blk_end; g0 += B) {
        Group G;
        G.col_begin = g0;
        G.col_end = std::min(blk_end, g0 + B);
        G.launch_begin = launches.size();
        size_t maxp = 0;
        for (int col = G.col_begin; col < G.col_end; ++col) maxp = std::max(maxp, plan.cols[col].passes.size());
        for (size_t t = 0; t < maxp; ++t) {
            Launch L;
            L.item_begin = (uint32_t)items.size();
            L.task_begin = (uint32_t)tasks.size();
            uint64_t poff = 0;
            for (int col = G.col_begin; col < G.col_end; ++col) {
                const ColumnPlan &cp = plan.cols[col];
                if (t >= cp.passes.size()) continue;
                const int b = col - G.col_begin;
                const uint32_t pidx = (uint32_t)(plan.col_pass_begin[col] + (int64_t)t);
                const HostPass &hp = cp.passes[t];
                LaunchItem it{};
                it.tile_begin = L.total_tiles;
                it.pass = pidx;
                it.ntiles = tiles;
                it.partial_off = poff;
                it.regA = reg(b, 0);
                it.regB = xi_of(cp.s, b, 0);
                it.regC = W > 1 ? xi_of(cp.s, b, 1) : nullptr;
                it.regD = W > 2 ? xi_of(cp.s, b, 2) : nullptr;
                it.regE = W > 3 ? xi_of(cp.s, b, 3) : nullptr;
                items.push_back(it);
                ++L.n_items;
                L.total_tiles += tiles;
                if (states) {
                    // no reduce tasks: n_tasks counts the elements the pass carries
                    for (size_t k = 0; k < hp.slot_dest.size(); ++k)
                        if (hp.slot_dest[k] < c.P * c.P) {
                            ++elements;
                            ++L.n_tasks;
                        }
                    continue;
                }
                for (size_t k = 0; k < hp.slot_dest.size(); ++k) {
                    tasks.push_back(ReduceTask{poff + (uint64_t)k * tiles, tiles, hp.slot_dest[k]});
                    ++L.n_tasks;
                    if (hp.slot_dest[k] < c.P * c.P) ++elements;   // (the rest: T of in-sweep seeds)
                }
                poff += (uint64_t)hp.slot_dest.size() * tiles;
            }
            if (poff > fr.partial_elems) fail(QNG_E_DEVICE, "fused sweep: partial buffer too small (internal)");
            launches.push_back(L);
        }
        G.launch_end = launches.size();
        groups.push_back(G);
    }

    // ---- device images
    std::vector<double> mats((size_t)c.M * 8, 0.0), fmats((size_t)c.M * 8, 0.0);
    for (const Rot &r : c.rots) {
        const Mat2 &m = fwd[r.pos];
        double *d = &fmats[(size_t)r.pos * 8];
        d[0] = m.a.real(); d[1] = m.a.imag(); d[2] = m.b.real(); d[3] = m.b.imag();
        d[4] = m.c.real(); d[5] = m.c.imag(); d[6] = m.d.real(); d[7] = m.d.imag();
        const Shear sh = adjoint_shear(r.axis, adj[r.pos]);
        mats[(size_t)r.pos * 8 + 0] = sh.u;
        mats[(size_t)r.pos * 8 + 1] = sh.w;
        if (r.ctrl >= 0) {
            const PlaneRot pl = adjoint_plane(r.axis, adj[r.pos]);
            mats[(size_t)r.pos * 8 + 2] = pl.c;
            mats[(size_t)r.pos * 8 + 3] = pl.s;
        }
    }
    fill_fixed_shears(c, adj, mats);
    std::vector<float> mats32(mats.begin(), mats.end());
    char *p = buf.scratch;
    auto take = [&](size_t bytes) { char *o = p; p += align256(bytes + 64); return o; };
    double *d_mats = (double *)take(mats.size() * 8);
    float *d_mats32 = (float *)take(mats32.size() * 4);
    double *d_fmats = (double *)take(fmats.size() * 8);
    // the forward matrices negated, then -I (row M): a seed that finds psi
    // negated (by the forward plan's passes) applies one of them instead, so
    // that the derivative-state variant's kept states carry no sign of psi
    std::vector<double> nfmats(fmats.size() + 8);
    for (size_t k = 0; k < fmats.size(); ++k) nfmats[k] = -fmats[k];
    nfmats[fmats.size()] = -1.0;
    nfmats[fmats.size() + 6] = -1.0;
    double *d_nfmats = (double *)take(nfmats.size() * 8);
    const double *d_negI = d_nfmats + fmats.size();
    DevPass *d_passes = (DevPass *)take(plan.dev_passes.size() * sizeof(DevPass));
    DevOp *d_ops = (DevOp *)take(plan.dev_ops.size() * sizeof(DevOp));
    DevMap *d_maps = (DevMap *)take(plan.dev_maps.size() * sizeof(DevMap));
    LaunchItem *d_items = (LaunchItem *)take(items.size() * sizeof(LaunchItem));
    ReduceTask *d_tasks = (ReduceTask *)take(tasks.size() * sizeof(ReduceTask));
    // the forward register's way between block tops as tile passes (the
    // recurrence only): the gates' own shears, one item per pass on psi.  A
    // gate with cos(theta/2) < 0 is applied negated (as in the sweeps), so psi
    // may carry a sign; every product and T, E and the gradient are quadratic
    // in it, and psi is put right at the end of the metric phase.
    const SweepPlan *fp = plan.forward ? plan.forward.get() : nullptr;
    std::vector<double> fshear;
    std::vector<LaunchItem> fitems;
    std::vector<uint8_t> seg_neg;
    double *d_fsh = nullptr;
    float *d_fsh32 = nullptr;
    DevPass *d_fpasses = nullptr;
    DevOp *d_fops = nullptr;
    DevMap *d_fmaps = nullptr;
    LaunchItem *d_fitems = nullptr;
    if (fp) {
        fshear.assign((size_t)c.M * 8, 0.0);
        std::vector<uint8_t> neg((size_t)c.M, 0);
        for (int pos = 0; pos < c.M; ++pos) {
            const int kind = c.gates[pos].kind;
            if (kind > QNG_RZ) continue;
            const int axis = kind == QNG_RX ? AX_X : kind == QNG_RY ? AX_Y : AX_Z;
            const Shear sh = adjoint_shear(axis, fwd[pos]);
            fshear[(size_t)pos * 8 + 0] = sh.u;
            fshear[(size_t)pos * 8 + 1] = sh.w;
            neg[pos] = fwd[pos].a.real() < 0;
        }
        int from = c.rots[0].pos;
        for (const ColumnPlan &cp : fp->cols) {
            uint8_t parity = 0;
            for (int k = from; k < c.rots[cp.s].pos; ++k) parity ^= neg[k];
            seg_neg.push_back(parity);
            from = c.rots[cp.s].pos;
        }
        for (size_t t = 0; t < fp->dev_passes.size(); ++t) {
            LaunchItem it{};
            it.pass = (uint32_t)t;
            it.ntiles = tiles;
            it.regA = state(0);
            fitems.push_back(it);
        }
        d_fsh = (double *)take(fshear.size() * 8);
        d_fsh32 = (float *)take(fshear.size() * 4);
        d_fpasses = (DevPass *)take(fp->dev_passes.size() * sizeof(DevPass));
        d_fops = (DevOp *)take(fp->dev_ops.size() * sizeof(DevOp));
        d_fmaps = (DevMap *)take(fp->dev_maps.size() * sizeof(DevMap));
        d_fitems = (LaunchItem *)take(fitems.size() * sizeof(LaunchItem));
    }
    std::vector<float> fshear32(fshear.begin(), fshear.end());
    double *d_partials = (double *)p;
    if ((size_t)(p - buf.scratch) + fr.partial_elems * 16 > buf.scratch_bytes)
        fail(QNG_E_DEVICE, "fused sweep: scratch too small (internal)");
    if (!mats.empty()) {
        FCHECK(hipMemcpyAsync(d_mats, mats.data(), mats.size() * 8, hipMemcpyHostToDevice, st));
        FCHECK(hipMemcpyAsync(d_mats32, mats32.data(), mats32.size() * 4, hipMemcpyHostToDevice, st));
        FCHECK(hipMemcpyAsync(d_fmats, fmats.data(), fmats.size() * 8, hipMemcpyHostToDevice, st));
        FCHECK(hipMemcpyAsync(d_nfmats, nfmats.data(), nfmats.size() * 8, hipMemcpyHostToDevice, st));
    }
    if (!plan.dev_passes.empty())
        FCHECK(hipMemcpyAsync(d_passes, plan.dev_passes.data(), plan.dev_passes.size() * sizeof(DevPass),
                              hipMemcpyHostToDevice, st));
    if (!plan.dev_ops.empty())
        FCHECK(hipMemcpyAsync(d_ops, plan.dev_ops.data(), plan.dev_ops.size() * sizeof(DevOp), hipMemcpyHostToDevice,
                              st));
    if (!plan.dev_maps.empty())
        FCHECK(hipMemcpyAsync(d_maps, plan.dev_maps.data(), plan.dev_maps.size() * sizeof(DevMap),
                              hipMemcpyHostToDevice, st));
    if (!items.empty())
        FCHECK(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(LaunchItem), hipMemcpyHostToDevice, st));
    if (!tasks.empty())
        FCHECK(hipMemcpyAsync(d_tasks, tasks.data(), tasks.size() * sizeof(ReduceTask), hipMemcpyHostToDevice, st));
    if (fp) {
        FCHECK(hipMemcpyAsync(d_fsh, fshear.data(), fshear.size() * 8, hipMemcpyHostToDevice, st));
        FCHECK(hipMemcpyAsync(d_fsh32, fshear32.data(), fshear32.size() * 4, hipMemcpyHostToDevice, st));
        if (!fp->dev_passes.empty()) {
            FCHECK(hipMemcpyAsync(d_fpasses, fp->dev_passes.data(), fp->dev_passes.size() * sizeof(DevPass),
                                  hipMemcpyHostToDevice, st));
            FCHECK(hipMemcpyAsync(d_fops, fp->dev_ops.data(), fp->dev_ops.size() * sizeof(DevOp),
                                  hipMemcpyHostToDevice, st));
            FCHECK(hipMemcpyAsync(d_fmaps, fp->dev_maps.data(), fp->dev_maps.size() * sizeof(DevMap),
                                  hipMemcpyHostToDevice, st));
            FCHECK(hipMemcpyAsync(d_fitems, fitems.data(), fitems.size() * sizeof(LaunchItem), hipMemcpyHostToDevice,
                                  st));
        }
    }
    FCHECK(hipStreamSynchronize(st));   // host vectors are released at return

    // ---- profiling events
    std::vector<hipEvent_t> ev;
    if (profile) {
        ev.resize(2 * launches.size());
        for (auto &e : ev) FCHECK(hipEventCreate(&e));
    }

    // ---- execute
    void *psi = state(0);
    int pos = 0;
    // A controlled rotation r has the diagonal element <y_r|(|1><1| on its
    // control)|y_r> (Sec. 2) instead of a constant: taken once, wherever psi
    // holds y_r (at its column's seed, or just before the forward pass applies it).
    std::vector<uint8_t> diag_done((size_t)c.P, 0);
    auto control_diag = [&](int r) {
        const Rot &rr = c.rots[r];
        if (rr.ctrl < 0 || diag_done[r]) return;
        launch_pauli_prod<R>(psi, psi, n, rr.ctrl, -1, buf.reduce_partials, buf.lraw + 2 * ((size_t)r * c.P + r), st,
                             rr.ctrl);
        stats->other_launches += 2;
        diag_done[r] = 1;
    };
    // forward gates up to `target`; a run of three or more CNOTs goes through
    // `scratch` (a register free at this point) as one gather and one copy
    auto forward_to = [&](int target, void *scratch) {
        for (; pos < target; ++pos) {
            const qng_gate &g = c.gates[pos];
            if (g.kind >= QNG_CRX && g.kind <= QNG_CRZ) {
                control_diag(c.rot_at[pos]);
                launch_apply_c1q<R>(psi, nullptr, n, g.q0, g.q1, to_dev(fwd[pos]), st);
                ++stats->other_launches;
                continue;
            }
            if (scratch && g.kind == QNG_CNOT) {
                int ctl[kCnotRunMax], tgt[kCnotRunMax], k = 0;
                while (pos + k < target && k < kCnotRunMax && c.gates[pos + k].kind == QNG_CNOT) {
                    ctl[k] = c.gates[pos + k].q0;
                    tgt[k] = c.gates[pos + k].q1;
                    ++k;
                }
                if (k >= 3) {
                    launch_cnot_run<R>(psi, scratch, n, ctl, tgt, k, st);
                    launch_copy<R>(scratch, psi, n, st);
                    stats->other_launches += 2;
                    pos += k - 1;
                    continue;
                }
            }
            if (g.kind == QNG_CNOT) launch_cnot<R>(psi, nullptr, n, g.q0, g.q1, st);
            else if (g.kind == QNG_CZ) launch_cz<R>(psi, nullptr, n, g.q0, g.q1, st);
            else launch_apply_1q<R>(psi, nullptr, n, g.q0, to_dev(fwd[pos]), st);
            ++stats->other_launches;
        }
    };
    forward_to(c.rots[0].pos, nullptr);
    if (states) {
        // the sweeps end in the frame just after rotation 0 (its adjoint is never
        // applied): lambda* = R_0 y_0 there, and column 0's derivative state is
        // sigma_0 lambda* (R_0 commutes with sigma_0)
        const Rot &r0 = c.rots[0];
        if (r0.ctrl >= 0) {
            // a controlled rotation 0: its diagonal at y_0, then the gate, and
            // column 0's state K_0 lambda* (K_0 commutes with the gate)
            control_diag(0);
            launch_apply_c1q<R>(psi, nullptr, n, r0.ctrl, r0.qubit, to_dev(fwd[r0.pos]), st);
            launch_seed<R>(psi, buf.xi, buf.xi + V, n, r0.qubit, r0.axis, st, r0.ctrl);
        } else {
            launch_advance_seed<R>(psi, buf.xi, buf.xi + V, n, r0.qubit, d_fmats + (size_t)r0.pos * 8, r0.qubit,
                                   r0.axis, buf.reduce_partials, buf.traw, st);
        }
        pos = r0.pos + 1;
    } else {
        launch_pauli_prod<R>(psi, psi, n, c.rots[0].qubit, c.rots[0].axis, buf.reduce_partials, buf.traw, st,
                             c.rots[0].ctrl);
        control_diag(0);
    }
    stats->other_launches += 2;
    uint8_t psi_negated = 0;
    // segment k of the forward plan takes psi from the top of block k - 1 (from
    // rotation 0 for k = 0) to the top of block k; psi is at the start of
    // segment at_seg (the derivative-state variant has applied rotation 0 of
    // segment 0 already)
    int at_seg = 0;
    // the first rotation a seed applies to psi (row of the forward table), or
    // -I when psi is negated and the seed applies none: the derivative-state
    // variant's kept states must not carry psi's sign
    auto seed_row = [&](int gate_pos) -> const double * {
        const bool fix = states && psi_negated;
        if (fix) psi_negated = 0;
        if (gate_pos < 0) return fix ? d_negI : d_fmats;
        return (fix ? d_nfmats : d_fmats) + (size_t)gate_pos * 8;
    };
    for (const Group &G : groups) {
        for (int col = G.col_begin; col < G.col_end; ++col) {
            const int s = plan.cols[col].s;    // top column of the block
            const Rot &rs = c.rots[s];
            const Rot &rp = c.rots[s - 1];
            const int b = col - G.col_begin;
            const int seg_next = col + 1;     // psi leaves the seed at the start of this segment
            // y_s = R_{s-1} y_{s-1} when rotation s-1 is the only gate in between:
            // one pass advances psi, seeds the top column and takes T_s (the
            // lower columns of a block are seeded inside its sweep).  When the
            // gate before rotation s-1 is a rotation too, on a third qubit, the
            // same pass applies both.
            if (rs.ctrl >= 0 || rp.ctrl >= 0) {
                // a controlled rotation at either end: the forward pass applies
                // every gate up to y_s, then the column is seeded with its generator
                forward_to(rs.pos, reg(b, 0));
                launch_seed<R>(psi, reg(b, 0), xi_of(s, b, W - 1), n, rs.qubit, rs.axis, st, rs.ctrl);
                launch_pauli_prod<R>(psi, psi, n, rs.qubit, rs.axis, buf.reduce_partials, buf.traw + 2 * s, st,
                                     rs.ctrl);
                control_diag(s);
                stats->other_launches += 3;
                at_seg = seg_next;
                continue;
            }
            const int ra = pos < c.M ? c.rot_at[pos] : -1;
            if (ra >= 0 && c.rots[ra].ctrl < 0 && pos + 1 == rp.pos && rs.pos == rp.pos + 1 && n >= 3 &&
                c.rots[ra].qubit != rp.qubit && c.rots[ra].qubit != rs.qubit && rp.qubit != rs.qubit) {
                launch_advance2_seed<R>(psi, reg(b, 0), xi_of(s, b, W - 1), n, c.rots[ra].qubit, seed_row(pos),
                                        rp.qubit, d_fmats + (size_t)rp.pos * 8, rs.qubit, rs.axis,
                                        buf.reduce_partials, buf.traw + 2 * s, st);
                stats->other_launches += 2;
                pos = rs.pos;
                at_seg = seg_next;
                continue;
            }
            // (the derivative-state variant is past the start of segment 0)
            if (fp && !(pos == rp.pos && rs.pos == rp.pos + 1) && !(states && col == 0)) {
                // more than the one rotation before the top: the gates up to the
                // top rotation in the forward plan's passes (usually one segment;
                // the first block of a later chunk of the derivative-state
                // variant is several segments on, and the rest of segment 0 runs
                // gate by gate), then lambda = psi = y_s, phi = sigma_s y_s and
                // T_s in one pass
                if (at_seg == 0 && states) {
                    forward_to(c.rots[plan.cols[0].s].pos, reg(b, 0));
                    at_seg = 1;
                }
                for (; at_seg <= col; ++at_seg) {
                    const int64_t t0 = fp->col_pass_begin[at_seg];
                    const int64_t t1 =
                        at_seg + 1 < (int)fp->cols.size() ? fp->col_pass_begin[at_seg + 1] : fp->total_passes;
                    for (int64_t t = t0; t < t1; ++t) {
                        launch_sweep_pass_states<R>(d_fitems + t, 1, tiles, d_fpasses, d_fops, d_fmaps, d_fsh,
                                                    d_fsh32, fp->m, fp->rb, 0, st);
                        ++stats->other_launches;
                    }
                    psi_negated ^= seg_neg[at_seg];
                }
                pos = rs.pos;
                const double *mrow = seed_row(-1);
                launch_advance_seed<R>(psi, reg(b, 0), xi_of(s, b, W - 1), n, mrow == d_negI ? rs.qubit : -1, mrow,
                                       rs.qubit, rs.axis, buf.reduce_partials, buf.traw + 2 * s, st);
                stats->other_launches += 2;
                continue;
            }
            forward_to(rp.pos, reg(b, 0));
            int qr = -1;
            const double *mrow = nullptr;
            if (rs.pos == rp.pos + 1 && pos == rp.pos) {   // (the states variant has applied rotation 0 already)
                qr = rp.qubit;
                mrow = seed_row(rp.pos);
                pos = rs.pos;
            } else {
                forward_to(rs.pos, reg(b, 0));
                mrow = seed_row(-1);
                if (mrow == d_negI) qr = rs.qubit;
            }
            launch_advance_seed<R>(psi, reg(b, 0), xi_of(s, b, W - 1), n, qr, mrow, rs.qubit, rs.axis,
                                   buf.reduce_partials, buf.traw + 2 * s, st);
            stats->other_launches += 2;
            at_seg = seg_next;
        }
        for (size_t li = G.launch_begin; li < G.launch_end; ++li) {
            const Launch &L = launches[li];
            if (profile) FCHECK(hipEventRecord(ev[2 * li], st));
            if (states)
                launch_sweep_pass_states<R>(d_items + L.item_begin, (int)L.n_items, L.total_tiles, d_passes, d_ops,
                                            d_maps, d_mats, d_mats32, plan.m, plan.rb, W, st, plan.ctrl);
            else
                launch_sweep_pass<R>(d_items + L.item_begin, (int)L.n_items, L.total_tiles, d_passes, d_ops, d_maps,
                                     d_mats, d_mats32, d_partials, plan.m, plan.rb, reg_mode, W, st, real_products,
                                     plan.ctrl);
            if (profile) FCHECK(hipEventRecord(ev[2 * li + 1], st));
            ++stats->sweep_launches;
            stats->sweep_tiles += L.total_tiles;
            stats->sweep_bytes += (double)L.n_items * 2.0 * (W + 1) * (double)V;
            if (states) {
                // the adjoint rotations on the phi registers (6) and on lambda,
                // shared by the block (6 / W), per amplitude per element
                stats->sweep_flops += (6.0 + 6.0 / W) * (double)L.n_tasks * (double)((uint64_t)1 << n);
                continue;
            }
            launch_reduce_tasks(d_tasks + L.task_begin, (int)L.n_tasks, d_partials, buf.lraw, st);
            ++stats->other_launches;
            stats->sweep_flops +=
                sweep_flops_per_amp(W, real_products) * (double)L.n_tasks * (double)((uint64_t)1 << n);
        }
    }
    if (psi_negated) {
        launch_apply_1q<R>(psi, nullptr, n, 0, DevMat2{-1, 0, 0, 0, 0, 0, -1, 0}, st);
        ++stats->other_launches;
    }
    stats->elements += elements;
    if (profile) {
        FCHECK(hipStreamSynchronize(st));
        double tot = 0.0;
        for (size_t li = 0; li < launches.size(); ++li) {
            float ms = 0.f;
            FCHECK(hipEventElapsedTime(&ms, ev[2 * li], ev[2 * li + 1]));
            tot += ms;
        }
        stats->sweep_ms += tot;
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
    return pos;
}

std::vector<StateChunk> state_chunks(const SweepPlan &plan, int max_cols) {
    const int W = plan.width;
    std::vector<StateChunk> out;
    int prev_hi = 0;
    for (int k = 0; k < (int)plan.cols.size(); ++k) {
        const int hi = plan.cols[k].s, lo = std::max(1, hi - W + 1);
        if (lo != prev_hi + 1) fail(QNG_E_DEVICE, "derivative states: column blocks out of order (internal)");
        prev_hi = hi;
        if (hi - lo + 1 > max_cols)
            fail(QNG_E_OUT_OF_MEMORY, "derivative states: a block of " + std::to_string(hi - lo + 1) +
                                          " columns does not fit in a chunk of " + std::to_string(max_cols));
        if (out.empty() || hi - out.back().col_lo + 1 > max_cols) out.push_back(StateChunk{k, k, lo, hi});
        out.back().blk_end = k + 1;
        out.back().col_hi = hi;
    }
    return out;
}

size_t kept_states(int P, int max_cols) {
    const int all = P - 1;
    return max_cols >= all ? (size_t)all + 3 : 2 * (size_t)max_cols + 3;
}

size_t states_gram_bytes(int n, int P, int max_cols) {
    const int all = P - 1;
    const int cmax = std::min(max_cols, all);
    // the largest of the calls' buffers (a smaller operand may take more chunks
    // of K): the shape depends on the operands' tile counts alone
    size_t b = 0;
    for (int t = 1; t <= (2 + cmax + 63) / 64; ++t) b = std::max(b, gram_partial_bytes(n, 64 * t, 0));
    if (cmax < all)
        for (int ta = 1; ta <= (cmax + 63) / 64; ++ta)
            for (int tb = 1; tb <= (cmax + 63) / 64; ++tb) b = std::max(b, gram_partial_bytes(n, 64 * ta, 64 * tb));
    return align256(b + 64) + align256((size_t)P + 1 + 64);
}

template <typename R>
int run_states_metric(const SweepPlan &plan, const FusedRun &fr, const Circuit &c, const std::vector<Mat2> &fwd,
                      const std::vector<Mat2> &adj, const FusedBuffers &buf, int max_cols,
                      const std::function<void()> &restart, hipStream_t st, qng_stats *stats, bool profile,
                      bool real_products) {
    const size_t V = buf.state_bytes;
    const int W = plan.width;
    const std::vector<StateChunk> ch = state_chunks(plan, max_cols);
    const int K = (int)ch.size();
    // The sign each kept state carries.  A rotation whose adjoint has
    // cos(theta/2) < 0 is applied negated to every register of a sweep
    // (circuit.hpp, adjoint_shear), which cancels in the recurrence's products
    // but not between states of different blocks.  In the block with top
    // column s, lambda (seeded unsigned at y_s) and the top phi register pass
    // through the adjoints of rotations s-1 .. 1; a lower column s_b is seeded
    // from lambda just after the adjoint of rotation s_b, so it carries the
    // signs of rotations s-1 .. s_b from lambda and those of s_b - 1 .. 1
    // after: every register of the block ends with the product of the signs of
    // rotations 1 .. s-1.  lambda* and column 0's state carry none.  Indexed
    // by column + 1.
    // (a controlled rotation's adjoint is applied as an exact plane rotation:
    // no sign)
    std::vector<int8_t> prefix((size_t)c.P + 1, 1);   // prefix[s]: signs of rotations 1 .. s-1
    for (int s = 2; s <= c.P; ++s) {
        const Rot &r = c.rots[s - 1];
        prefix[s] = (int8_t)(r.ctrl < 0 && adj[r.pos].a.real() < 0 ? -prefix[s - 1] : prefix[s - 1]);
    }
    std::vector<int8_t> signs((size_t)c.P + 1, 1);
    for (const ColumnPlan &cp : plan.cols)
        for (int k = 0; k < W; ++k) {
            const int col = cp.s - (W - 1) + k;
            if (col >= 1) signs[1 + col] = prefix[cp.s];
        }
    FCHECK(hipMemcpyAsync(buf.gram_signs, signs.data(), signs.size(), hipMemcpyHostToDevice, st));
    FCHECK(hipStreamSynchronize(st));   // `signs` is released at return
    stats->state_chunks = K;

    const bool c64 = sizeof(R) == 4;
    int cmax = 0;
    for (const StateChunk &k : ch) cmax = std::max(cmax, k.col_hi - k.col_lo + 1);
    char *ra = buf.xi + 2 * V;             // the chunk whose own products are taken next
    char *rb = ra + (size_t)cmax * V;      // the chunks paired with it
    int pos = 0;
    bool first = true;
    auto ncol = [&](int k) { return ch[k].col_hi - ch[k].col_lo + 1; };
    auto prep = [&](int k, char *region) {
        if (!first) restart();
        first = false;
        FusedBuffers b = buf;
        b.blk_begin = ch[k].blk_begin;
        b.blk_end = ch[k].blk_end;
        b.xi_chunk = region;
        b.chunk_col0 = ch[k].col_lo;
        pos = run_fused_metric<R>(plan, fr, c, fwd, adj, b, st, stats, profile, 0, real_products);
    };
    // Re (and, for the complex G, Im) of the inner products, on the matrix cores
    auto gram = [&](const GramSet &A, const GramSet *B) {
        for (int mode = 0; mode < (real_products ? 1 : 2); ++mode) {
            launch_gram(A, B, c64, c.n, c.P, mode, buf.gram_signs, buf.gram_partials, buf.lraw, buf.traw, st);
            stats->other_launches += 2;
        }
    };
    // lambda*, column 0 and chunk k among themselves
    auto own = [&](int k, char *region) {
        GramSet A;
        A.p1 = buf.xi;
        A.n1 = 2;
        A.p2 = region;
        A.n = 2 + ncol(k);
        A.col1 = -1;
        A.col2 = ch[k].col_lo;
        gram(A, nullptr);
    };
    auto chunk_set = [&](int k, char *region) {
        GramSet S;
        S.p1 = region;
        S.n1 = S.n = ncol(k);
        S.col1 = ch[k].col_lo;
        return S;
    };
    // The top chunk first; chunk i is paired with every chunk below it, the
    // lowest first, so that the last one prepared (chunk i - 1) is the next to
    // take its own products: 1 + K (K - 1) / 2 preparations in all, the
    // repeated ones those of the lower chunks, whose sweeps are the shorter.
    // The forward state is left where the last preparation leaves it (pos).
    prep(K - 1, ra);
    own(K - 1, ra);
    for (int i = K - 1; i > 0; --i) {
        for (int j = 0; j < i; ++j) {
            prep(j, rb);
            const GramSet A = chunk_set(j, rb), B = chunk_set(i, ra);
            gram(A, &B);
        }
        std::swap(ra, rb);
        own(i - 1, ra);
    }
    return pos;
}

size_t fused_gradient_scratch_bytes(const SweepPlan &g, int M) {
    size_t b = 0;
    b += align256((size_t)M * 64 + 64);
    b += align256((size_t)M * 32 + 64);
    b += align256(g.dev_passes.size() * sizeof(DevPass) + 64);
    b += align256(g.dev_ops.size() * sizeof(DevOp) + 64);
    b += align256(g.dev_maps.size() * sizeof(DevMap) + 64);
    b += align256(g.dev_passes.size() * sizeof(LaunchItem) + 64);
    b += align256((size_t)(g.P + 1) * sizeof(ReduceTask) + 64);
    b += align256((size_t)g.max_slots * ((size_t)1 << (g.n - g.m)) * 16 + 64);
    return b;
}

template <typename R>
void run_fused_gradient(const SweepPlan &g, const Circuit &c, const std::vector<Mat2> &adj, void *lam, void *psi,
                        double *graw, char *scratch, size_t scratch_bytes, hipStream_t st, qng_stats *stats,
                        bool profile, int reg_mode) {
    if (g.cols.empty()) return;
    const ColumnPlan &cp = g.cols[0];
    const uint32_t tiles = 1u << (c.n - g.m);
    std::vector<LaunchItem> items;
    std::vector<ReduceTask> tasks;
    std::vector<uint32_t> task_begin;
    for (size_t t = 0; t < cp.passes.size(); ++t) {
        LaunchItem it{};
        it.tile_begin = 0;
        it.pass = (uint32_t)t;
        it.ntiles = tiles;
        it.partial_off = 0;
        it.regA = lam;
        it.regB = psi;
        items.push_back(it);
        task_begin.push_back((uint32_t)tasks.size());
        for (size_t k = 0; k < cp.passes[t].slot_dest.size(); ++k)
            tasks.push_back(ReduceTask{(uint64_t)k * tiles, tiles, cp.passes[t].slot_dest[k]});
    }
    task_begin.push_back((uint32_t)tasks.size());
    std::vector<double> mats((size_t)c.M * 8, 0.0);
    for (const Rot &r : c.rots) {
        const Shear sh = adjoint_shear(r.axis, adj[r.pos]);
        mats[(size_t)r.pos * 8 + 0] = sh.u;
        mats[(size_t)r.pos * 8 + 1] = sh.w;
        if (r.ctrl >= 0) {
            const PlaneRot pl = adjoint_plane(r.axis, adj[r.pos]);
            mats[(size_t)r.pos * 8 + 2] = pl.c;
            mats[(size_t)r.pos * 8 + 3] = pl.s;
        }
    }
    fill_fixed_shears(c, adj, mats);
    std::vector<float> mats32(mats.begin(), mats.end());
    char *p = scratch;
    auto take = [&](size_t bytes) { char *o = p; p += align256(bytes + 64); return o; };
    double *d_mats = (double *)take(mats.size() * 8);
    float *d_mats32 = (float *)take(mats32.size() * 4);
    DevPass *d_passes = (DevPass *)take(g.dev_passes.size() * sizeof(DevPass));
    DevOp *d_ops = (DevOp *)take(g.dev_ops.size() * sizeof(DevOp));
    DevMap *d_maps = (DevMap *)take(g.dev_maps.size() * sizeof(DevMap));
    LaunchItem *d_items = (LaunchItem *)take(items.size() * sizeof(LaunchItem));
    ReduceTask *d_tasks = (ReduceTask *)take(tasks.size() * sizeof(ReduceTask));
    double *d_partials = (double *)p;
    if ((size_t)(p - scratch) + (size_t)g.max_slots * tiles * 16 > scratch_bytes)
        fail(QNG_E_DEVICE, "fused gradient: scratch too small (internal)");
    auto put = [&](void *dst, const void *src, size_t bytes) {
        if (bytes) FCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    };
    put(d_mats, mats.data(), mats.size() * 8);
    put(d_mats32, mats32.data(), mats32.size() * 4);
    put(d_passes, g.dev_passes.data(), g.dev_passes.size() * sizeof(DevPass));
    put(d_ops, g.dev_ops.data(), g.dev_ops.size() * sizeof(DevOp));
    put(d_maps, g.dev_maps.data(), g.dev_maps.size() * sizeof(DevMap));
    put(d_items, items.data(), items.size() * sizeof(LaunchItem));
    put(d_tasks, tasks.data(), tasks.size() * sizeof(ReduceTask));
    FCHECK(hipStreamSynchronize(st));   // host vectors are released at return
    std::vector<hipEvent_t> ev;
    if (profile) {
        ev.resize(2 * items.size());
        for (auto &e : ev) FCHECK(hipEventCreate(&e));
    }
    const size_t V = ((size_t)1 << c.n) * 2 * sizeof(R);
    for (size_t t = 0; t < items.size(); ++t) {
        if (profile) FCHECK(hipEventRecord(ev[2 * t], st));
        launch_sweep_pass<R>(d_items + t, 1, tiles, d_passes, d_ops, d_maps, d_mats, d_mats32, d_partials, g.m, g.rb,
                             reg_mode, 1, st, false, g.ctrl);
        if (profile) FCHECK(hipEventRecord(ev[2 * t + 1], st));
        const uint32_t nt = task_begin[t + 1] - task_begin[t];
        launch_reduce_tasks(d_tasks + task_begin[t], (int)nt, d_partials, graw, st);
        ++stats->sweep_launches;
        ++stats->other_launches;
        stats->sweep_tiles += tiles;
        stats->sweep_bytes += 4.0 * (double)V;
        stats->sweep_flops += 20.0 * (double)nt * (double)((uint64_t)1 << c.n);
    }
    if (profile) {
        FCHECK(hipStreamSynchronize(st));
        for (size_t t = 0; t < items.size(); ++t) {
            float ms = 0.f;
            FCHECK(hipEventElapsedTime(&ms, ev[2 * t], ev[2 * t + 1]));
            stats->sweep_ms += ms;
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
}

template void run_fused_gradient<double>(const SweepPlan &, const Circuit &, const std::vector<Mat2> &, void *, void *,
                                         double *, char *, size_t, hipStream_t, qng_stats *, bool, int);
template void run_fused_gradient<float>(const SweepPlan &, const Circuit &, const std::vector<Mat2> &, void *, void *,
                                        double *, char *, size_t, hipStream_t, qng_stats *, bool, int);

template int run_fused_metric<double>(const SweepPlan &, const FusedRun &, const Circuit &, const std::vector<Mat2> &,
                                      const std::vector<Mat2> &, const FusedBuffers &, hipStream_t, qng_stats *, bool, int,
                                      bool);
template int run_fused_metric<float>(const SweepPlan &, const FusedRun &, const Circuit &, const std::vector<Mat2> &,
                                     const std::vector<Mat2> &, const FusedBuffers &, hipStream_t, qng_stats *, bool, int,
                                     bool);

template int run_states_metric<double>(const SweepPlan &, const FusedRun &, const Circuit &, const std::vector<Mat2> &,
                                       const std::vector<Mat2> &, const FusedBuffers &, int,
                                       const std::function<void()> &, hipStream_t, qng_stats *, bool, bool);
template int run_states_metric<float>(const SweepPlan &, const FusedRun &, const Circuit &, const std::vector<Mat2> &,
                                      const std::vector<Mat2> &, const FusedBuffers &, int,
                                      const std::function<void()> &, hipStream_t, qng_stats *, bool, bool);

}  // namespace qng
