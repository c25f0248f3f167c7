// batch.cpp -- schedule and executor of the batched metric (see batch.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <numeric>
#include <string>

#include "batch.hpp"
#include "kernels.hpp"

namespace qng {

namespace {

#define BCHECK(call)                                                                                  \
    do {                                                                                              \
        hipError_t _e = (call);                                                                       \
        if (_e != hipSuccess) fail(QNG_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr uint64_t kSeedBlocksMax = 1024;   // work-groups per seed in a round (the rest by grid stride)

struct ImageLayout {
    size_t passes, ops, maps, items, tasks, seed_items, seed_tasks, total;
};

ImageLayout image_layout(const BatchSchedule &s) {
    ImageLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes + 64); return o; };
    L.passes = take(s.passes.size() * sizeof(DevPass));
    L.ops = take(s.ops.size() * sizeof(DevOp));
    L.maps = take(s.maps.size() * sizeof(DevMap));
    L.items = take(s.items.size() * sizeof(LaunchItem));
    L.tasks = take(s.tasks.size() * sizeof(ReduceTask));
    L.seed_items = take(s.seeds.size() * sizeof(SeedItem));
    L.seed_tasks = take(s.seed_tasks.size() * sizeof(ReduceTask));
    L.total = off;
    return L;
}

}  // namespace

BatchSchedule build_batch_schedule(const std::vector<const Circuit *> &members,
                                   const std::vector<std::shared_ptr<const SweepPlan>> &plans, int amp,
                                   const BatchTuning &tun, uint64_t arena_cap) {
    BatchSchedule S;
    const int nb = (int)members.size();
    S.amp = amp;
    S.plans = plans;
    S.gate_base.resize(nb);
    S.lraw_base.resize(nb);
    std::vector<int64_t> pass_base(nb);
    for (int b = 0; b < nb; ++b) {
        const Circuit &c = *members[b];
        const SweepPlan &p = *plans[b];
        if (b == 0) {
            S.m = p.m;
            S.rb = p.rb;
            S.width = p.width;
            S.ctrl = false;
        } else if (p.m != S.m || p.rb != S.rb || p.width != S.width) {
            fail(QNG_E_DEVICE, "batch schedule: members of one class differ in tile or block width (internal)");
        }
        S.ctrl = S.ctrl || p.ctrl;
        pass_base[b] = (int64_t)S.passes.size();
        const uint32_t op_base = (uint32_t)S.ops.size(), map_base = (uint32_t)S.maps.size();
        S.gate_base[b] = S.mat_rows;
        S.mat_rows += c.M;
        S.lraw_base[b] = S.lraw_elems;
        S.lraw_elems += (int64_t)c.P * c.P + c.P;
        for (DevPass dp : p.dev_passes) {
            dp.op_begin += op_base;
            dp.map_load += map_base;
            S.passes.push_back(dp);
        }
        for (DevOp op : p.dev_ops) {
            if (op.type == OPC_XPOSE) op.aux += (int32_t)map_base;
            if (op.gate >= 0) op.gate += (int32_t)S.gate_base[b];
            S.ops.push_back(op);
        }
        S.maps.insert(S.maps.end(), p.dev_maps.begin(), p.dev_maps.end());
        if (c.P == 1) S.singles.push_back(b);
        S.elements += (int64_t)c.P * (c.P - 1) / 2;
    }
    if (S.lraw_elems > INT32_MAX) fail(QNG_E_INVALID_ARG, "batch too large: more than 2^31 metric entries");

    // queue: members in increasing register size, then depth; columns in increasing s
    std::vector<int> order(nb);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (members[a]->n != members[b]->n) return members[a]->n < members[b]->n;
        return members[a]->P < members[b]->P;
    });
    std::vector<std::pair<int, int>> queue;
    for (int b : order)
        for (int col = 0; col < (int)plans[b]->cols.size(); ++col) queue.emplace_back(b, col);

    struct Active {
        int b, col;
        size_t t;
        uint64_t reg;
    };
    std::map<int, std::vector<uint64_t>> free_pairs;   // by register size (qubits)
    uint64_t bump = 0, act_tiles = 0;
    std::vector<Active> act;
    size_t qi = 0;
    const uint64_t target = (uint64_t)std::max(1, tun.target_tiles);
    for (;;) {
        BatchLaunch L{};
        L.prep_begin = (uint32_t)S.preps.size();
        while (qi < queue.size()) {
            const int b = queue[qi].first, col = queue[qi].second;
            const int n = members[b]->n;
            const uint64_t tiles = uint64_t(1) << (n - S.m);
            const uint64_t pair = (uint64_t)(S.width + 1) * ((uint64_t(1) << n) * (uint64_t)amp);
            if (!act.empty() && act_tiles + tiles > target) break;
            uint64_t reg;
            std::vector<uint64_t> &fl = free_pairs[n];
            if (!fl.empty()) {
                reg = fl.back();
                fl.pop_back();
            } else if (act.empty() || bump + pair <= arena_cap) {
                reg = bump;
                bump += pair;
            } else {
                break;
            }
            S.preps.push_back(BatchPrep{b, col, reg});
            act.push_back(Active{b, col, 0, reg});
            act_tiles += tiles;
            ++qi;
        }
        if (act.empty()) break;
        L.n_preps = (uint32_t)S.preps.size() - L.prep_begin;
        L.item_begin = (uint32_t)S.items.size();
        L.task_begin = (uint32_t)S.tasks.size();
        uint64_t poff = 0;
        for (const Active &a : act) {
            const SweepPlan &p = *plans[a.b];
            const HostPass &hp = p.cols[a.col].passes[a.t];
            const int n = members[a.b]->n;
            const uint32_t tiles = 1u << (n - S.m);
            LaunchItem it{};
            it.tile_begin = L.total_tiles;
            it.pass = (uint32_t)(pass_base[a.b] + p.col_pass_begin[a.col] + (int64_t)a.t);
            it.ntiles = tiles;
            it.partial_off = poff;
            const uint64_t V = (uint64_t(1) << n) * (uint64_t)amp;
            it.regA = (void *)(uintptr_t)a.reg;
            it.regB = (void *)(uintptr_t)(a.reg + V);
            it.regC = S.width > 1 ? (void *)(uintptr_t)(a.reg + 2 * V) : nullptr;
            it.regD = S.width > 2 ? (void *)(uintptr_t)(a.reg + 3 * V) : nullptr;
            it.regE = S.width > 3 ? (void *)(uintptr_t)(a.reg + 4 * V) : nullptr;
            S.items.push_back(it);
            ++L.n_items;
            L.total_tiles += tiles;
            for (size_t k = 0; k < hp.slot_dest.size(); ++k) {
                S.tasks.push_back(ReduceTask{poff + (uint64_t)k * tiles, tiles,
                                             (int32_t)(S.lraw_base[a.b] + hp.slot_dest[k])});
                ++L.n_tasks;
            }
            poff += (uint64_t)hp.slot_dest.size() * tiles;
        }
        S.partial_elems = std::max(S.partial_elems, poff);
        S.launches.push_back(L);
        std::vector<Active> next;
        next.reserve(act.size());
        for (Active a : act) {
            ++a.t;
            if (a.t < plans[a.b]->cols[a.col].passes.size()) {
                next.push_back(a);
            } else {
                const int n = members[a.b]->n;
                free_pairs[n].push_back(a.reg);
                act_tiles -= uint64_t(1) << (n - S.m);
            }
        }
        act.swap(next);
    }
    S.arena_bytes = bump;

    // the seeds of every launch in rounds, the forward registers' positions
    // followed as the executor moves them
    std::vector<int> fpos(nb, -1);
    for (BatchLaunch &L : S.launches) {
        L.round_begin = (uint32_t)S.rounds.size();
        std::map<int, int> seen;
        std::vector<int> ridx(L.n_preps);
        int nr = 0;
        for (uint32_t k = 0; k < L.n_preps; ++k) {
            ridx[k] = seen[S.preps[L.prep_begin + k].member]++;
            nr = std::max(nr, ridx[k] + 1);
        }
        for (int r = 0; r < nr; ++r) {
            BatchRound R{(uint32_t)S.seeds.size(), 0, 0, 0};
            // the one kernel's items first (registers of >= 3 qubits, no controlled
            // rotation at the seed), then the seeds run on their own
            auto multi = [&](uint32_t k) {
                const BatchPrep &pr = S.preps[L.prep_begin + k];
                const Circuit &c = *members[pr.member];
                const int sidx = plans[pr.member]->cols[pr.col].s;
                return c.n >= 3 && c.rots[sidx].ctrl < 0 && c.rots[sidx - 1].ctrl < 0;
            };
            for (int big = 1; big >= 0; --big)
            for (uint32_t k = 0; k < L.n_preps; ++k) {
                if (ridx[k] != r || multi(k) != (big == 1)) continue;
                const BatchPrep &pr = S.preps[L.prep_begin + k];
                const Circuit &c = *members[pr.member];
                const int sidx = plans[pr.member]->cols[pr.col].s;
                const Rot &rs = c.rots[sidx];
                const Rot &rp = c.rots[sidx - 1];
                int &p = fpos[pr.member];
                if (p < 0) p = c.rots[0].pos;
                BatchSeed sd{};
                sd.member = pr.member;
                sd.fwd_to = -1;
                sd.qa = sd.qb = sd.pa = sd.pb = -1;
                sd.qs = rs.qubit;
                sd.axis = rs.axis;
                sd.s = sidx;
                sd.lam_off = pr.reg_off;
                sd.phi_off = pr.reg_off + (uint64_t)S.width * (uint64_t(1) << c.n) * (uint64_t)amp;
                const int ra = p < c.M ? c.rot_at[p] : -1;
                if (rs.ctrl >= 0 || rp.ctrl >= 0) {
                    sd.fwd_to = rs.pos;          // every gate up to y_s, then the generator's seed
                    sd.ctrl = 1;
                } else if (ra >= 0 && c.rots[ra].ctrl < 0 && p + 1 == rp.pos && rs.pos == rp.pos + 1 && c.n >= 3 &&
                           c.rots[ra].qubit != rp.qubit && c.rots[ra].qubit != rs.qubit && rp.qubit != rs.qubit) {
                    sd.qa = c.rots[ra].qubit;   // two rotations before y_s
                    sd.pa = p;
                    sd.qb = rp.qubit;
                    sd.pb = rp.pos;
                } else if (rs.pos == rp.pos + 1) {
                    sd.fwd_to = rp.pos;          // the gates up to rotation s - 1, then that rotation
                    sd.qa = rp.qubit;
                    sd.pa = rp.pos;
                } else {
                    sd.fwd_to = rs.pos;          // every gate up to y_s
                }
                p = rs.pos;
                if (c.n >= 3 && !sd.ctrl) {
                    const uint64_t groups = uint64_t(1) << (c.n - 3);
                    sd.nblocks = (uint32_t)std::min<uint64_t>(kSeedBlocksMax, (groups + 255) / 256);
                    sd.block_begin = R.total_blocks;
                    R.total_blocks += sd.nblocks;
                    S.seed_tasks.push_back(ReduceTask{(uint64_t)sd.block_begin, sd.nblocks,
                                                      (int32_t)(S.lraw_base[pr.member] + (int64_t)c.P * c.P + sidx)});
                    ++R.n_multi;
                } else {
                    sd.nblocks = 0;   // seeded on its own; its task is never launched
                    S.seed_tasks.push_back(ReduceTask{0, 0, 0});
                }
                S.seeds.push_back(sd);
                ++R.n_seeds;
            }
            S.partial_elems = std::max<uint64_t>(S.partial_elems, R.total_blocks);
            S.rounds.push_back(R);
        }
        L.n_rounds = (uint32_t)nr;
    }
    S.partial_elems += 16;
    return S;
}

size_t batch_image_bytes(const BatchSchedule &s) { return image_layout(s).total; }

void upload_batch_images(const BatchSchedule &s, const BatchDevice &d, hipStream_t st) {
    const ImageLayout L = image_layout(s);
    std::vector<LaunchItem> items = s.items;
    for (LaunchItem &it : items) {
        it.regA = d.arena + (uintptr_t)it.regA;
        it.regB = d.arena + (uintptr_t)it.regB;
        if (s.width > 1) it.regC = d.arena + (uintptr_t)it.regC;
        if (s.width > 2) it.regD = d.arena + (uintptr_t)it.regD;
        if (s.width > 3) it.regE = d.arena + (uintptr_t)it.regE;
    }
    auto put = [&](size_t off, const void *src, size_t bytes) {
        if (bytes) BCHECK(hipMemcpyAsync(d.images + off, src, bytes, hipMemcpyHostToDevice, st));
    };
    put(L.passes, s.passes.data(), s.passes.size() * sizeof(DevPass));
    put(L.ops, s.ops.data(), s.ops.size() * sizeof(DevOp));
    put(L.maps, s.maps.data(), s.maps.size() * sizeof(DevMap));
    put(L.items, items.data(), items.size() * sizeof(LaunchItem));
    put(L.tasks, s.tasks.data(), s.tasks.size() * sizeof(ReduceTask));
    std::vector<SeedItem> seeds(s.seeds.size());
    for (size_t k = 0; k < s.seeds.size(); ++k) {
        const BatchSeed &sd = s.seeds[k];
        SeedItem &it = seeds[k];
        it.psi = d.psi[sd.member];
        it.lam = d.arena + sd.lam_off;
        it.phi = d.arena + sd.phi_off;
        it.ma = sd.qa >= 0 ? d.fwd_mats + (s.gate_base[sd.member] + sd.pa) * 8 : nullptr;
        it.mb = sd.qb >= 0 ? d.fwd_mats + (s.gate_base[sd.member] + sd.pb) * 8 : nullptr;
        it.qa = sd.qa;
        it.qb = sd.qb;
        it.qs = sd.qs;
        it.axis = sd.axis;
        it.n = s.plans[sd.member]->n;
        it.block_begin = sd.block_begin;
        it.nblocks = sd.nblocks;
    }
    put(L.seed_items, seeds.data(), seeds.size() * sizeof(SeedItem));
    put(L.seed_tasks, s.seed_tasks.data(), s.seed_tasks.size() * sizeof(ReduceTask));
    BCHECK(hipStreamSynchronize(st));   // `items` and `seeds` are released at return
}

int batch_final_pos(const Circuit &c) { return c.P ? c.rots[c.P - 1].pos : 0; }

template <typename R>
void enqueue_batch_metric(const BatchSchedule &s, const std::vector<const Circuit *> &members, const BatchDevice &d,
                          int reg_mode, hipStream_t st, std::vector<hipEvent_t> *events, bool real_products) {
    const ImageLayout IL = image_layout(s);
    const DevPass *passes = (const DevPass *)(d.images + IL.passes);
    const DevOp *ops = (const DevOp *)(d.images + IL.ops);
    const DevMap *maps = (const DevMap *)(d.images + IL.maps);
    const LaunchItem *items = (const LaunchItem *)(d.images + IL.items);
    const ReduceTask *tasks = (const ReduceTask *)(d.images + IL.tasks);
    const int nb = (int)members.size();
    std::vector<int> pos(nb, 0);
    std::vector<char> started(nb, 0);
    std::vector<std::vector<uint8_t>> diag_done(nb);

    // A controlled rotation r has the diagonal element <y_r|(|1><1| on its
    // control)|y_r> (Sec. 2) instead of a constant: taken once, where the
    // forward register of its member holds y_r.
    auto control_diag = [&](int b, int r) {
        const Circuit &c = *members[b];
        const Rot &rr = c.rots[r];
        if (rr.ctrl < 0) return;
        if (diag_done[b].empty()) diag_done[b].assign((size_t)c.P, 0);
        if (diag_done[b][r]) return;
        diag_done[b][r] = 1;
        launch_pauli_prod<R>(d.psi[b], d.psi[b], c.n, rr.ctrl, -1, d.reduce_partials,
                             d.lraw + 2 * (s.lraw_base[b] + (int64_t)r * c.P + r), st, rr.ctrl);
    };

    // forward gates of member b up to `target`; with a scratch register free,
    // a run of three or more CNOTs is one gather and one copy back
    auto forward_to = [&](int b, int target, void *scratch) {
        const Circuit &c = *members[b];
        for (; pos[b] < target; ++pos[b]) {
            const qng_gate &g = c.gates[pos[b]];
            if (scratch && g.kind == QNG_CNOT) {
                int ctl[kCnotRunMax], tgt[kCnotRunMax], k = 0;
                while (pos[b] + k < target && k < kCnotRunMax && c.gates[pos[b] + k].kind == QNG_CNOT) {
                    ctl[k] = c.gates[pos[b] + k].q0;
                    tgt[k] = c.gates[pos[b] + k].q1;
                    ++k;
                }
                if (k >= 3) {
                    launch_cnot_run<R>(d.psi[b], scratch, c.n, ctl, tgt, k, st);
                    launch_copy<R>(scratch, d.psi[b], c.n, st);
                    pos[b] += k - 1;
                    continue;
                }
            }
            if (g.kind == QNG_CNOT) {
                launch_cnot<R>(d.psi[b], nullptr, c.n, g.q0, g.q1, st);
            } else if (g.kind == QNG_CZ) {
                launch_cz<R>(d.psi[b], nullptr, c.n, g.q0, g.q1, st);
            } else if (g.kind >= QNG_CRX && g.kind <= QNG_CRZ) {
                control_diag(b, c.rot_at[pos[b]]);   // (q0 the control, q1 the target)
                launch_apply_c1q_tab<R>(d.psi[b], nullptr, c.n, g.q0, g.q1,
                                        d.fwd_mats + (s.gate_base[b] + pos[b]) * 8, st);
            } else {
                launch_apply_1q_tab<R>(d.psi[b], nullptr, c.n, g.q0, d.fwd_mats + (s.gate_base[b] + pos[b]) * 8, st);
            }
        }
    };
    auto start = [&](int b) {
        if (started[b]) return;
        started[b] = 1;
        const Circuit &c = *members[b];
        forward_to(b, c.rots[0].pos, nullptr);
        launch_pauli_prod<R>(d.psi[b], d.psi[b], c.n, c.rots[0].qubit, c.rots[0].axis, d.reduce_partials, d.traw[b],
                             st, c.rots[0].ctrl);
        control_diag(b, 0);
    };
    for (int b : s.singles) start(b);
    const SeedItem *seed_items = (const SeedItem *)(d.images + IL.seed_items);
    const ReduceTask *seed_tasks = (const ReduceTask *)(d.images + IL.seed_tasks);
    for (size_t li = 0; li < s.launches.size(); ++li) {
        const BatchLaunch &L = s.launches[li];
        for (uint32_t r = L.round_begin; r < L.round_begin + L.n_rounds; ++r) {
            // a round: the gates its seeds need first (one kernel per gate), then
            // all its seeds in one kernel and their T in one reduction
            const BatchRound &rd = s.rounds[r];
            for (uint32_t k = rd.seed_begin; k < rd.seed_begin + rd.n_seeds; ++k) {
                const BatchSeed &sd = s.seeds[k];
                start(sd.member);
                char *lam = d.arena + sd.lam_off;
                if (sd.fwd_to >= 0) forward_to(sd.member, sd.fwd_to, lam);
                if (sd.ctrl) {
                    // a controlled rotation at either end: psi = y_s, seeded with the generator
                    const Circuit &c = *members[sd.member];
                    const Rot &rs = c.rots[sd.s];
                    launch_seed<R>(d.psi[sd.member], lam, d.arena + sd.phi_off, c.n, rs.qubit, rs.axis, st, rs.ctrl);
                    launch_pauli_prod<R>(d.psi[sd.member], d.psi[sd.member], c.n, rs.qubit, rs.axis, d.reduce_partials,
                                         d.traw[sd.member] + 2 * sd.s, st, rs.ctrl);
                    control_diag(sd.member, sd.s);
                } else if (sd.nblocks == 0) {
                    // a register below 3 qubits: seeded on its own
                    const Circuit &c = *members[sd.member];
                    const double *mrow = sd.qa >= 0 ? d.fwd_mats + (s.gate_base[sd.member] + sd.pa) * 8 : d.fwd_mats;
                    launch_advance_seed<R>(d.psi[sd.member], lam, d.arena + sd.phi_off, c.n, sd.qa, mrow, sd.qs,
                                            sd.axis, d.reduce_partials, d.traw[sd.member] + 2 * sd.s, st);
                }
                pos[sd.member] = members[sd.member]->rots[sd.s].pos;
            }
            if (rd.n_multi) {
                launch_seed_multi<R>(seed_items + rd.seed_begin, (int)rd.n_multi, rd.total_blocks, d.partials, st);
                launch_reduce_tasks(seed_tasks + rd.seed_begin, (int)rd.n_multi, d.partials, d.lraw, st);
            }
        }
        if (events) BCHECK(hipEventRecord((*events)[2 * li], st));
        launch_sweep_pass<R>(items + L.item_begin, (int)L.n_items, L.total_tiles, passes, ops, maps, d.adj_mats,
                             d.adj_mats32, d.partials, s.m, s.rb, reg_mode, s.width, st, real_products, s.ctrl);
        if (events) BCHECK(hipEventRecord((*events)[2 * li + 1], st));
        launch_reduce_tasks(tasks + L.task_begin, (int)L.n_tasks, d.partials, d.lraw, st);
    }
}

template void enqueue_batch_metric<double>(const BatchSchedule &, const std::vector<const Circuit *> &,
                                           const BatchDevice &, int, hipStream_t, std::vector<hipEvent_t> *, bool);
template void enqueue_batch_metric<float>(const BatchSchedule &, const std::vector<const Circuit *> &,
                                          const BatchDevice &, int, hipStream_t, std::vector<hipEvent_t> *, bool);

}  // namespace qng
