// sweep.cpp -- planner and host executor of the fused, tiled sweep passes.
// See sweep.hpp for the model.
#include "sweep.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>

namespace qng {

namespace {

enum : uint8_t { TY_X = 0, TY_Y = 1, TY_Z = 2 };
enum : uint8_t { EV_PROD = 0, EV_UNAPPLY = 1 };

struct Event {
    uint8_t kind;
    uint8_t nq;
    uint8_t type[2];
    int q[2];
    int pos;   // gate position (UNAPPLY) / position of the rotation (PROD)
    int rot;   // rotation index (PROD), -1 otherwise
    int gkind; // gate kind (UNAPPLY)
};

Event unapply_event(const Circuit &c, int pos) {
    const qng_gate &g = c.gates[pos];
    Event e{};
    e.kind = EV_UNAPPLY;
    e.pos = pos;
    e.rot = -1;
    e.gkind = g.kind;
    switch (g.kind) {
    case QNG_RX: e.nq = 1; e.q[0] = g.q0; e.type[0] = TY_X; break;
    case QNG_RY: e.nq = 1; e.q[0] = g.q0; e.type[0] = TY_Y; break;
    case QNG_RZ: e.nq = 1; e.q[0] = g.q0; e.type[0] = TY_Z; break;
    case QNG_CNOT: e.nq = 2; e.q[0] = g.q0; e.type[0] = TY_Z; e.q[1] = g.q1; e.type[1] = TY_X; break;
    default: e.nq = 2; e.q[0] = g.q0; e.type[0] = TY_Z; e.q[1] = g.q1; e.type[1] = TY_Z; break;
    }
    return e;
}

Event prod_event(const Circuit &c, int r) {
    Event e{};
    e.kind = EV_PROD;
    e.nq = 1;
    e.q[0] = c.rots[r].qubit;
    e.type[0] = (uint8_t)c.rots[r].axis;   // AX_X/AX_Y/AX_Z == TY_X/TY_Y/TY_Z
    e.pos = c.rots[r].pos;
    e.rot = r;
    e.gkind = -1;
    return e;
}

// Backward sweep of column s: positions rots[s].pos-1 down to rots[0].pos; the
// inner product of rotation r comes just before the adjoint of rotation r (the
// adjoint of the first rotation is never needed).
std::vector<Event> column_events(const Circuit &c, int s) {
    std::vector<Event> ev;
    const int p0 = c.rots[0].pos;
    for (int k = c.rots[s].pos - 1; k >= p0; --k) {
        const int r = c.rot_at[k];
        if (r >= 0) {
            ev.push_back(prod_event(c, r));
            if (k > p0) ev.push_back(unapply_event(c, k));
        } else {
            ev.push_back(unapply_event(c, k));
        }
    }
    return ev;
}

bool executable(const Event &e, const std::vector<uint8_t> &in_tile) {
    if (e.kind == EV_PROD) return e.type[0] == TY_Z || in_tile[e.q[0]];
    switch (e.gkind) {
    case QNG_CNOT: return in_tile[e.q[1]];
    case QNG_CZ: return in_tile[e.q[0]] || in_tile[e.q[1]];
    default: return in_tile[e.q[0]];
    }
}

// One in-order scan: emit every pending event that is ready (no earlier pending
// event it fails to commute with) and executable in the tile.  Returns the
// number emitted; if `out` is given, the emitted indices are appended and the
// events marked done.
int scan(const std::vector<Event> &ev, std::vector<uint8_t> &done, const std::vector<int> &pending,
         const std::vector<uint8_t> &in_tile, int n, std::vector<int> *out) {
    std::vector<int> cnt((size_t)n * 3, 0);
    int emitted = 0, slots = 0;
    for (int idx : pending) {
        if (done[idx]) continue;
        const Event &e = ev[idx];
        bool ready = true;
        for (int j = 0; j < e.nq && ready; ++j) {
            const int *cq = &cnt[(size_t)e.q[j] * 3];
            for (int t = 0; t < 3; ++t)
                if (t != e.type[j] && cq[t]) { ready = false; break; }
        }
        bool ok = ready && executable(e, in_tile);
        if (ok && e.kind == EV_PROD) {
            if (slots >= kMaxSlots) ok = false;
            else ++slots;
        }
        if (ok) {
            ++emitted;
            if (out) {
                out->push_back(idx);
                done[idx] = 1;
            }
        } else {
            for (int j = 0; j < e.nq; ++j) ++cnt[(size_t)e.q[j] * 3 + e.type[j]];
        }
    }
    return emitted;
}

int choose_and_emit(const std::vector<Event> &ev, std::vector<uint8_t> &done, std::vector<int> &pending, int n, int m,
                    int carriers, std::vector<uint8_t> &tile_out, std::vector<int> &emitted) {
    std::vector<uint8_t> in_tile(n, 0);
    if (n <= m) {
        std::fill(in_tile.begin(), in_tile.end(), 1);
    } else {
        const int w = m - carriers;
        int best = -1;
        std::vector<uint8_t> best_tile;
        auto consider = [&](const std::vector<uint8_t> &cand) {
            const int sc = scan(ev, done, pending, cand, n, nullptr);
            if (sc > best) { best = sc; best_tile = cand; }
        };
        // candidate 1: carriers + qubits of the first ready-but-blocked events
        {
            std::vector<uint8_t> cand(n, 0);
            for (int q = 0; q < carriers; ++q) cand[q] = 1;
            std::vector<int> cnt((size_t)n * 3, 0);
            int added = 0;
            for (int idx : pending) {
                if (done[idx] || added >= w) continue;
                const Event &e = ev[idx];
                bool ready = true;
                for (int j = 0; j < e.nq && ready; ++j)
                    for (int t = 0; t < 3; ++t)
                        if (t != e.type[j] && cnt[(size_t)e.q[j] * 3 + t]) { ready = false; break; }
                if (ready && !executable(e, cand)) {
                    const int need = (e.kind == EV_UNAPPLY && e.gkind == QNG_CNOT) ? e.q[1] : e.q[0];
                    if (!cand[need]) { cand[need] = 1; ++added; }
                }
                for (int j = 0; j < e.nq; ++j) ++cnt[(size_t)e.q[j] * 3 + e.type[j]];
            }
            consider(cand);
        }
        // candidates 2..: carriers + a window of consecutive qubits
        for (int a = carriers; a + w <= n; ++a) {
            std::vector<uint8_t> cand(n, 0);
            for (int q = 0; q < carriers; ++q) cand[q] = 1;
            for (int q = a; q < a + w; ++q) cand[q] = 1;
            consider(cand);
        }
        in_tile = best_tile;
        // every pass of a plan has exactly m tile qubits: the launch covers 2^(n-m) tiles
        int have = 0;
        for (int q = 0; q < n; ++q) have += in_tile[q];
        for (int q = 0; q < n && have < m; ++q)
            if (!in_tile[q]) { in_tile[q] = 1; ++have; }
    }
    emitted.clear();
    const int k = scan(ev, done, pending, in_tile, n, &emitted);
    if (k == 0) fail(QNG_E_DEVICE, "sweep planner made no progress (internal error)");
    tile_out.clear();
    for (int q = 0; q < n; ++q)
        if (in_tile[q]) tile_out.push_back((uint8_t)q);
    if ((int)tile_out.size() != std::min(n, m)) fail(QNG_E_DEVICE, "sweep planner: tile of wrong size (internal)");
    // drop finished events from the pending list
    std::vector<int> keep;
    keep.reserve(pending.size());
    for (int idx : pending)
        if (!done[idx]) keep.push_back(idx);
    pending.swap(keep);
    return k;
}

HostPass make_pass(const Circuit &c, int s, const std::vector<Event> &ev, const std::vector<int> &emitted,
                   const std::vector<uint8_t> &tile) {
    HostPass hp;
    hp.tile = tile;
    std::vector<int> local(c.n, -1);
    for (size_t b = 0; b < tile.size(); ++b) local[tile[b]] = (int)b;
    for (size_t k = 0; k < emitted.size(); ++k) {
        const Event &e = ev[emitted[k]];
        DevOp op{};
        op.b0 = op.b1 = kNoBit;
        op.gate = -1;
        if (e.kind == EV_PROD) {
            const int q = e.q[0];
            const uint16_t slot = (uint16_t)hp.slot_dest.size();
            hp.slot_dest.push_back((int32_t)(e.rot * c.P + s));
            op.slot = slot;
            op.axis = e.type[0];
            op.q0 = (uint8_t)q;
            if (local[q] < 0) {
                op.type = OP_ZSUM;
            } else {
                op.b0 = (uint8_t)local[q];
                // fuse with the adjoint of the same rotation when it follows immediately
                if (k + 1 < emitted.size()) {
                    const Event &f = ev[emitted[k + 1]];
                    if (f.kind == EV_UNAPPLY && f.pos == e.pos) {
                        op.type = OP_PRODROT;
                        op.gate = f.pos;
                        hp.ops.push_back(op);
                        ++k;
                        continue;
                    }
                }
                op.type = OP_PROD;
            }
        } else {
            const qng_gate &g = c.gates[e.pos];
            op.gate = e.pos;
            if (g.kind == QNG_CNOT) {
                op.type = OP_CNOT;
                op.q0 = (uint8_t)g.q0;
                op.b0 = local[g.q0] < 0 ? kNoBit : (uint8_t)local[g.q0];
                op.b1 = (uint8_t)local[g.q1];
            } else if (g.kind == QNG_CZ) {
                op.type = OP_CZ;
                op.q0 = (uint8_t)g.q0;
                op.q1 = (uint8_t)g.q1;
                op.b0 = local[g.q0] < 0 ? kNoBit : (uint8_t)local[g.q0];
                op.b1 = local[g.q1] < 0 ? kNoBit : (uint8_t)local[g.q1];
            } else {
                op.type = OP_ROT;
                op.b0 = (uint8_t)local[g.q0];
                op.q0 = (uint8_t)g.q0;
            }
        }
        hp.ops.push_back(op);
    }
    return hp;
}

}  // namespace

int default_tile_qubits(int n, int amp_bytes) {
    const int m = amp_bytes >= 16 ? 11 : 12;
    return n < m ? n : m;
}

SweepPlan build_sweep_plan(const Circuit &c, int tile_qubits, int amp_bytes, int /*small*/) {
    SweepPlan plan;
    plan.n = c.n;
    plan.P = c.P;
    int m = tile_qubits > 0 ? tile_qubits : default_tile_qubits(c.n, amp_bytes);
    if (m > kMaxTileQubits) m = kMaxTileQubits;
    if (m > c.n) m = c.n;
    plan.m = m;
    plan.carriers = c.n > m ? std::min(amp_bytes >= 16 ? 3 : 4, m - 1) : 0;
    if (c.n > m && m - plan.carriers < 2) fail(QNG_E_INVALID_ARG, "tile too small for the carrier qubits");
    for (int s = 1; s < c.P; ++s) {
        ColumnPlan cp;
        cp.s = s;
        std::vector<Event> ev = column_events(c, s);
        std::vector<uint8_t> done(ev.size(), 0);
        std::vector<int> pending(ev.size());
        for (size_t i = 0; i < ev.size(); ++i) pending[i] = (int)i;
        std::vector<uint8_t> tile;
        std::vector<int> emitted;
        while (!pending.empty()) {
            choose_and_emit(ev, done, pending, c.n, m, plan.carriers, tile, emitted);
            cp.passes.push_back(make_pass(c, s, ev, emitted, tile));
        }
        plan.cols.push_back(std::move(cp));
    }
    // flatten
    for (const ColumnPlan &cp : plan.cols) {
        plan.col_pass_begin.push_back((int64_t)plan.dev_passes.size());
        for (const HostPass &hp : cp.passes) {
            DevPass dp{};
            dp.op_begin = (uint32_t)plan.dev_ops.size();
            dp.n_ops = (uint32_t)hp.ops.size();
            dp.n_slots = (uint16_t)hp.slot_dest.size();
            dp.m = (uint8_t)hp.tile.size();
            dp.n = (uint8_t)c.n;
            for (size_t b = 0; b < hp.tile.size(); ++b) dp.tile_q[b] = hp.tile[b];
            std::vector<uint8_t> in(c.n, 0);
            for (uint8_t q : hp.tile) in[q] = 1;
            int k = 0;
            for (int q = 0; q < c.n; ++q)
                if (!in[q]) dp.rest_q[k++] = (uint8_t)q;
            dp.nrest = (uint8_t)k;
            for (const DevOp &op : hp.ops) {
                if (op.type == OP_ZSUM) dp.has_zsum = 1;
                plan.dev_ops.push_back(op);
            }
            plan.dev_passes.push_back(dp);
            plan.max_slots = std::max<int64_t>(plan.max_slots, dp.n_slots);
            for (const DevOp &op : hp.ops)
                if (op.type == OP_CNOT) { ++plan.load_maps; break; }
        }
    }
    plan.total_passes = (int64_t)plan.dev_passes.size();
    plan.total_ops = (int64_t)plan.dev_ops.size();
    return plan;
}

size_t SweepPlan::device_bytes() const {
    return dev_passes.size() * sizeof(DevPass) + dev_ops.size() * sizeof(DevOp);
}

void SweepPlan::fill_info(qng_plan_info *out) const {
    out->passes = total_passes;
    out->elements = (int64_t)P * (P - 1) / 2;
    out->ops = total_ops;
    out->load_maps = load_maps;
    out->tile_qubits = m;
    out->small_n = n <= m ? 1 : 0;
}

const SweepPlan &SweepCache::get(const Circuit &c, int tile_qubits, int amp_bytes, int small) {
    std::vector<int32_t> key = {c.n, c.M, c.P, tile_qubits, amp_bytes, small};
    for (const qng_gate &g : c.gates) {
        key.push_back(g.kind);
        key.push_back(g.q0);
        key.push_back(g.q1);
        key.push_back(g.param >= 0 ? 1 : 0);
    }
    auto it = plans.find(key);
    if (it != plans.end()) return *it->second;
    if (plans.size() > 16) plans.clear();
    auto p = std::make_shared<SweepPlan>(build_sweep_plan(c, tile_qubits, amp_bytes, small));
    plans[key] = p;
    return *p;
}

FusedRun fused_config(const SweepPlan &plan, int requested_streams, size_t state_bytes, size_t free_bytes) {
    FusedRun fr;
    const int64_t tiles = int64_t(1) << (plan.n - plan.m);
    const int cols = (int)plan.cols.size();
    int B = requested_streams;
    if (B <= 0) {
        const int64_t target = 4096;   // work-groups per launch to fill 256 CUs several times over
        B = (int)std::max<int64_t>(1, (target + tiles - 1) / tiles);
    }
    if (B > cols) B = std::max(1, cols);
    // keep the column registers within a quarter of the free memory
    while (B > 1 && (size_t)(1 + 2 * B) * state_bytes > free_bytes / 4) --B;
    fr.B = B;
    fr.partial_elems = (size_t)B * (size_t)plan.max_slots * (size_t)tiles + 16;
    return fr;
}

}  // namespace qng
