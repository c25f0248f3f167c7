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
enum : uint8_t { EV_PROD = 0, EV_UNAPPLY = 1, EV_SEED = 2 };

struct Event {
    uint8_t kind;
    uint8_t nq;
    uint8_t type[2];
    int q[2];
    int pos;   // gate position (UNAPPLY) / position of the rotation (PROD, SEED)
    int rot;   // rotation index (PROD, SEED), -1 otherwise
    int gkind; // gate kind (UNAPPLY)
    int fa;    // PROD: first active phi register of the block (columns above the rotation)
    int sb;    // SEED: phi register seeded
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
    // controlled rotations: Z-type on the control q0, sigma-type on the target q1
    case QNG_CRX: e.nq = 2; e.q[0] = g.q0; e.type[0] = TY_Z; e.q[1] = g.q1; e.type[1] = TY_X; break;
    case QNG_CRY: e.nq = 2; e.q[0] = g.q0; e.type[0] = TY_Z; e.q[1] = g.q1; e.type[1] = TY_Y; break;
    case QNG_CRZ: e.nq = 2; e.q[0] = g.q0; e.type[0] = TY_Z; e.q[1] = g.q1; e.type[1] = TY_Z; break;
    default: e.nq = 2; e.q[0] = g.q0; e.type[0] = TY_Z; e.q[1] = g.q1; e.type[1] = TY_Z; break;
    }
    return e;
}

bool is_controlled_gate(int kind) { return kind == QNG_CRX || kind == QNG_CRY || kind == QNG_CRZ; }

Event prod_event(const Circuit &c, int r) {
    Event e{};
    e.kind = EV_PROD;
    e.nq = 1;
    e.q[0] = c.rots[r].qubit;
    e.type[0] = (uint8_t)c.rots[r].axis;   // AX_X/AX_Y/AX_Z == TY_X/TY_Y/TY_Z
    if (c.rots[r].ctrl >= 0) {             // generator |1><1|_c (x) sigma_t: Z-type on the control too
        e.nq = 2;
        e.q[1] = c.rots[r].ctrl;
        e.type[1] = TY_Z;
    }
    e.pos = c.rots[r].pos;
    e.rot = r;
    e.gkind = -1;
    return e;
}

// Seed of phi register b of a block where lambda reaches y_r (the state just
// before rotation r): phi_b = sigma_r lambda.  It acts on rotation r's qubit
// with sigma_r's type, like an inner product.
Event seed_event(const Circuit &c, int r, int b) {
    Event e = prod_event(c, r);
    e.kind = EV_SEED;
    e.sb = b;
    return e;
}

// Backward sweep of a block of columns s_b = s - width + 1 + b (b < width,
// s_b >= 1) sharing lambda: positions rots[s].pos-1 down to rots[0].pos.  The
// inner product of rotation r (for every column above r) comes just before the
// adjoint of rotation r (the adjoint of the first rotation is never needed);
// after the adjoint of a block column's own rotation lambda is y_{s_b}, and
// that column's phi register is seeded there.  With width 1 this is the sweep
// of column s alone (Sec. 3, Alg. 1 inner loop).
//
// rot_block (nullable, width 1 only): block id per rotation.  The column then
// takes the inner products of the rotations of its own block only and its
// sweep stops at the lowest of them (block-diagonal approximation of G); a
// column alone in its block below s has no events.
std::vector<Event> block_events(const Circuit &c, int s, int width, const std::vector<int> *rot_block) {
    std::vector<Event> ev;
    int lo = 0;
    if (rot_block) {
        lo = -1;
        for (int r = s - 1; r >= 0; --r)
            if ((*rot_block)[r] == (*rot_block)[s]) lo = r;
        if (lo < 0) return ev;
    }
    const int p0 = c.rots[lo].pos;
    const int s_first = s - width + 1;     // column of phi register 0 (may be < 1: absent)
    for (int k = c.rots[s].pos - 1; k >= p0; --k) {
        const int r = c.rot_at[k];
        if (r >= 0) {
            Event e = prod_event(c, r);
            e.fa = std::max(0, r + 1 - s_first);
            if (!rot_block || (*rot_block)[r] == (*rot_block)[s]) ev.push_back(e);
            if (k > p0) ev.push_back(unapply_event(c, k));
            if (r >= std::max(1, s_first) && r < s) ev.push_back(seed_event(c, r, r - s_first));
        } else {
            ev.push_back(unapply_event(c, k));
        }
    }
    return ev;
}

// Reverse sweep of the energy gradient: positions M-1 down to rots[0].pos,
// the inner product of every rotation r just before its adjoint (again never
// needed for the first rotation).
std::vector<Event> gradient_events(const Circuit &c) {
    std::vector<Event> ev;
    const int p0 = c.rots[0].pos;
    for (int k = c.M - 1; k >= p0; --k) {
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
    // an X/Y product or seed needs its target in the tile; a Z one runs on any
    // bit (outside the tile: a tile sum, or for a controlled one a sign from
    // the tile base); a control may lie anywhere
    if (e.kind == EV_PROD || e.kind == EV_SEED) return e.type[0] == TY_Z || in_tile[e.q[0]];
    switch (e.gkind) {
    case QNG_CNOT:
    case QNG_CRX:
    case QNG_CRY:
    case QNG_CRZ: return in_tile[e.q[1]];
    case QNG_CZ: return in_tile[e.q[0]] || in_tile[e.q[1]];
    default: return in_tile[e.q[0]];
    }
}

// Ordering state of an in-order scan: per qubit and Pauli type, the pending
// (not emitted) events seen so far, and the highest phi register whose seed is
// pending.  An event is ready when it commutes with every pending event before
// it, and an inner product also waits for the seeds of the phi registers it
// reads.
struct Blockers {
    std::vector<int> cnt;
    int seed_b = -1;
    explicit Blockers(int n) : cnt((size_t)n * 3, 0) {}
    bool ready(const Event &e) const {
        for (int j = 0; j < e.nq; ++j) {
            const int *cq = &cnt[(size_t)e.q[j] * 3];
            for (int t = 0; t < 3; ++t)
                if (t != e.type[j] && cq[t]) return false;
        }
        return !(e.kind == EV_PROD && e.fa <= seed_b);
    }
    void block(const Event &e) {
        for (int j = 0; j < e.nq; ++j) ++cnt[(size_t)e.q[j] * 3 + e.type[j]];
        if (e.kind == EV_SEED) seed_b = std::max(seed_b, e.sb);
    }
};

// Inner-product slots an event takes: one per active phi register, one for
// the T product of a seed.
int event_slots(const Event &e, int width) {
    if (e.kind == EV_PROD) return width - e.fa;
    return e.kind == EV_SEED ? 1 : 0;
}

// One in-order scan: emit every pending event that is ready (no earlier pending
// event it fails to commute with) and executable in the tile.  Returns the
// number emitted; if `out` is given, the emitted indices are appended and the
// events marked done.
int scan(const std::vector<Event> &ev, std::vector<uint8_t> &done, const std::vector<int> &pending,
         const std::vector<uint8_t> &in_tile, int n, int width, std::vector<int> *out) {
    Blockers bl(n);
    int emitted = 0, slots = 0;
    for (int idx : pending) {
        if (done[idx]) continue;
        const Event &e = ev[idx];
        bool ok = bl.ready(e) && executable(e, in_tile);
        const int need = event_slots(e, width);
        if (ok && need) {
            if (slots + need > kMaxSlots) ok = false;
            else slots += need;
        }
        if (ok) {
            ++emitted;
            if (out) {
                out->push_back(idx);
                done[idx] = 1;
            }
        } else {
            bl.block(e);
        }
    }
    return emitted;
}

int choose_and_emit(const std::vector<Event> &ev, std::vector<uint8_t> &done, std::vector<int> &pending, int n, int m,
                    int carriers, int width, std::vector<uint8_t> &tile_out, std::vector<int> &emitted) {
    std::vector<uint8_t> in_tile(n, 0);
    if (n <= m) {
        std::fill(in_tile.begin(), in_tile.end(), 1);
    } else {
        const int w = m - carriers;
        int best = -1;
        std::vector<uint8_t> best_tile;
        auto consider = [&](const std::vector<uint8_t> &cand) {
            const int sc = scan(ev, done, pending, cand, n, width, nullptr);
            if (sc > best) { best = sc; best_tile = cand; }
        };
        // candidate 1: carriers + qubits of the first ready-but-blocked events
        {
            std::vector<uint8_t> cand(n, 0);
            for (int q = 0; q < carriers; ++q) cand[q] = 1;
            Blockers bl(n);
            int added = 0;
            for (int idx : pending) {
                if (done[idx] || added >= w) continue;
                const Event &e = ev[idx];
                if (bl.ready(e) && !executable(e, cand)) {
                    const int need =
                        (e.kind == EV_UNAPPLY && (e.gkind == QNG_CNOT || is_controlled_gate(e.gkind))) ? e.q[1] : e.q[0];
                    if (!cand[need]) { cand[need] = 1; ++added; }
                }
                bl.block(e);
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
    const int k = scan(ev, done, pending, in_tile, n, width, &emitted);
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

// Local bit that an event needs in a register (X/Y rotations and inner
// products, CNOT targets), or -1 for diagonal events that run on any bit.
int needs_register(const Event &e, const std::vector<int> &local) {
    if (e.kind == EV_PROD || e.kind == EV_SEED) return e.type[0] == TY_Z ? -1 : local[e.q[0]];
    switch (e.gkind) {
    case QNG_RX:
    case QNG_RY: return local[e.q[0]];
    case QNG_CNOT:
    case QNG_CRX:
    case QNG_CRY: return local[e.q[1]];
    default: return -1;
    }
}

// In-order scan of the pass's events with a register set (bit mask over local
// bits): emit every ready event whose register need is met.
int scan_phase(const std::vector<Event> &ev, const std::vector<int> &pending, std::vector<uint8_t> &done,
               uint32_t regset, const std::vector<int> &local, int n, std::vector<int> *out) {
    Blockers bl(n);
    int emitted = 0;
    for (int idx : pending) {
        if (done[idx]) continue;
        const Event &e = ev[idx];
        const int need = needs_register(e, local);
        const bool ok = bl.ready(e) && (need < 0 || ((regset >> need) & 1u));
        if (ok) {
            ++emitted;
            if (out) {
                out->push_back(idx);
                done[idx] = 1;
            }
        } else {
            bl.block(e);
        }
    }
    return emitted;
}

DevMap mapping_for(uint32_t regset, int m, int rb, int carriers) {
    DevMap mp{};
    int p = 0;
    for (int b = 0; b < m; ++b)
        if ((regset >> b) & 1u) mp.pos[p++] = (uint8_t)b;
    for (int b = 0; b < carriers; ++b)
        if (!((regset >> b) & 1u)) mp.pos[p++] = (uint8_t)b;
    for (int b = carriers; b < m; ++b)
        if (!((regset >> b) & 1u)) mp.pos[p++] = (uint8_t)b;
    (void)rb;
    return mp;
}

uint8_t location(const DevMap &mp, int rb, int m, int localbit) {
    for (int p = 0; p < m; ++p)
        if (mp.pos[p] == localbit) return p < rb ? (uint8_t)p : (uint8_t)(kLocThread | (p - rb));
    return kLocBase;
}

// Destinations of a block's inner products: element (r, column of phi register
// b) -> r * stride + col0 + b (metric: r * P + s_b; gradient: r); the T product
// of a seeded column s_b -> t_base + s_b.
struct SlotDest {
    int stride, col0, t_base;
};

HostPass make_pass(const Circuit &c, const SlotDest &sd, const std::vector<Event> &ev, const std::vector<int> &emitted,
                   const std::vector<uint8_t> &tile, int rb, int carriers, int width) {
    HostPass hp;
    hp.tile = tile;
    hp.rb = rb;
    const int m = (int)tile.size();
    std::vector<int> local(c.n, -1);
    for (size_t b = 0; b < tile.size(); ++b) local[tile[b]] = (int)b;
    const uint32_t carrier_mask = (1u << carriers) - 1u;

    // ---- phases: greedy choice of the register set, then emission in scan order
    std::vector<uint8_t> done(ev.size(), 0);
    std::vector<int> pending = emitted;
    std::vector<std::pair<uint32_t, std::vector<int>>> phases;
    uint32_t current = 0;
    bool have_current = false;
    while (!pending.empty()) {
        std::vector<uint32_t> cands;
        if (have_current) cands.push_back(current);
        {   // registers for the first ready events that need one
            uint32_t rs = 0;
            int added = 0;
            Blockers bl(c.n);
            for (int idx : pending) {
                if (added >= rb) break;
                const Event &e = ev[idx];
                const int need = needs_register(e, local);
                if (bl.ready(e) && need >= 0 && !((rs >> need) & 1u)) { rs |= 1u << need; ++added; }
                bl.block(e);
            }
            for (int b = m - 1; b >= 0 && added < rb; --b)
                if (!((rs >> b) & 1u)) { rs |= 1u << b; ++added; }
            cands.push_back(rs);
        }
        for (int a = 0; a + rb <= m; ++a) cands.push_back(((1u << rb) - 1u) << a);
        int best = -1000000;
        uint32_t best_rs = cands[0];
        for (uint32_t rs : cands) {
            const int k = scan_phase(ev, pending, done, rs, local, c.n, nullptr);
            const int score = 4 * k - ((have_current && rs != current) ? 3 : 0);
            if (k > 0 && score > best) { best = score; best_rs = rs; }
        }
        std::vector<int> out;
        scan_phase(ev, pending, done, best_rs, local, c.n, &out);
        if (out.empty()) fail(QNG_E_DEVICE, "sweep planner: phase made no progress (internal error)");
        std::vector<int> keep;
        for (int idx : pending)
            if (!done[idx]) keep.push_back(idx);
        pending.swap(keep);
        if (have_current && best_rs == current) {
            phases.back().second.insert(phases.back().second.end(), out.begin(), out.end());
        } else {
            phases.push_back({best_rs, out});
            current = best_rs;
            have_current = true;
        }
    }

    // ---- thread mappings: load with the carriers on the lanes
    auto add_map = [&](const DevMap &mp) { hp.maps.push_back(mp); return (int)hp.maps.size() - 1; };
    uint32_t load_rs = phases[0].first;
    bool load_xpose = false;
    if (load_rs & carrier_mask) {
        load_rs = ((1u << rb) - 1u) << (m - rb);
        load_xpose = true;
    }
    hp.map_load = add_map(mapping_for(load_rs, m, rb, carriers));
    int cur_map = hp.map_load;
    auto xpose_to = [&](uint32_t rs) {
        const int k = add_map(mapping_for(rs, m, rb, carriers));
        DevOp op{};
        op.type = OP_XPOSE;
        op.b0 = op.b1 = kLocBase;
        op.gate = -1;
        op.aux = k;
        hp.ops.push_back(op);
        cur_map = k;
        ++hp.transposes;
    };

    for (size_t ph = 0; ph < phases.size(); ++ph) {
        if (ph > 0 || load_xpose) xpose_to(phases[ph].first);
        const DevMap &mp = hp.maps[cur_map];
        const std::vector<int> &order = phases[ph].second;
        auto loc_of_qubit = [&](int q) -> uint8_t { return local[q] < 0 ? kLocBase : location(mp, rb, m, local[q]); };
        for (size_t k = 0; k < order.size(); ++k) {
            const Event &e = ev[order[k]];
            DevOp op{};
            op.b0 = op.b1 = kLocBase;
            op.gate = -1;
            if (e.kind == EV_SEED) {
                const int q = e.q[0];
                op.type = e.nq == 2 ? OP_CSEED : OP_SEED;
                if (e.nq == 2) {
                    op.q1 = (uint8_t)e.q[1];
                    op.b1 = loc_of_qubit(e.q[1]);
                }
                op.slot = (uint16_t)hp.slot_dest.size();
                hp.slot_dest.push_back((int32_t)(sd.t_base + sd.col0 + e.sb));
                op.axis = e.type[0];
                op.q0 = (uint8_t)q;
                op.b0 = loc_of_qubit(q);
                op.aux = e.sb;
            } else if (e.kind == EV_PROD) {
                const int q = e.q[0];
                op.slot = (uint16_t)hp.slot_dest.size();
                for (int b = e.fa; b < width; ++b)
                    hp.slot_dest.push_back((int32_t)(e.rot * sd.stride + sd.col0 + b));
                op.aux = e.fa;
                op.axis = e.type[0];
                op.q0 = (uint8_t)q;
                const bool fuse = k + 1 < order.size() && ev[order[k + 1]].kind == EV_UNAPPLY &&
                                  ev[order[k + 1]].pos == e.pos;
                if (e.nq == 2) {
                    // controlled: target in the tile (executable), control anywhere
                    op.b0 = loc_of_qubit(q);
                    op.q1 = (uint8_t)e.q[1];
                    op.b1 = loc_of_qubit(e.q[1]);
                    if (e.type[0] == TY_Z) op.type = fuse ? OP_PRODCDIAG : OP_PRODCZ;
                    else op.type = fuse ? OP_PRODCROT : OP_PRODC;
                } else if (local[q] < 0) {
                    op.type = OP_ZSUM;
                } else if (e.type[0] == TY_Z) {
                    op.b0 = loc_of_qubit(q);
                    op.type = fuse ? OP_PRODDIAG : OP_PRODZ;
                } else {
                    op.b0 = loc_of_qubit(q);
                    op.type = fuse ? OP_PRODROT : OP_PROD;
                }
                if (fuse && op.type != OP_ZSUM) {
                    op.gate = ev[order[k + 1]].pos;
                    ++k;
                }
            } else {
                const qng_gate &g = c.gates[e.pos];
                op.gate = e.pos;
                op.q0 = (uint8_t)g.q0;
                if (g.kind == QNG_CNOT) {
                    op.type = OP_CNOT;
                    op.q1 = (uint8_t)g.q1;
                    op.b0 = loc_of_qubit(g.q1);       // a register position
                    op.b1 = loc_of_qubit(g.q0);
                } else if (g.kind == QNG_CZ) {
                    op.type = OP_CZ;
                    op.q1 = (uint8_t)g.q1;
                    op.b0 = loc_of_qubit(g.q0);
                    op.b1 = loc_of_qubit(g.q1);
                } else if (g.kind == QNG_RZ) {
                    op.type = OP_DIAG;
                    op.b0 = loc_of_qubit(g.q0);
                } else if (is_controlled_gate(g.kind)) {
                    op.type = g.kind == QNG_CRZ ? OP_CDIAG : OP_CROT;
                    op.axis = g.kind == QNG_CRX ? TY_X : g.kind == QNG_CRY ? TY_Y : TY_Z;
                    op.q0 = (uint8_t)g.q1;            // target
                    op.q1 = (uint8_t)g.q0;            // control
                    op.b0 = loc_of_qubit(g.q1);
                    op.b1 = loc_of_qubit(g.q0);
                } else {
                    op.type = OP_ROT;
                    op.axis = g.kind == QNG_RX ? TY_X : TY_Y;
                    op.b0 = loc_of_qubit(g.q0);
                }
            }
            hp.ops.push_back(op);
        }
    }
    // store with the carriers on the lanes
    if (current & carrier_mask) xpose_to(((1u << rb) - 1u) << (m - rb));
    return hp;
}

}  // namespace

int default_tile_qubits(int n, int amp_bytes, bool reg_f64) {
    // FP32 registers: 12 tile qubits (16 amplitudes of each register per
    // thread); FP64 registers: 11 (8 per thread), the most that fits the
    // register file without spills.  Wider tiles fuse more of each column
    // into one pass (measured at n = 26: 2363 passes at 12 qubits against 2718
    // at 11, at the same time per pass).
    const int m = (amp_bytes == 8 && !reg_f64) ? 12 : 11;
    return n < m ? n : m;
}

int register_bits(int m, int /*amp_bytes*/) {
    int rb = m - 8;
    if (rb < 2) rb = std::min(m, 2);
    return rb > 4 ? 4 : rb;
}

namespace {

// Tile width, register bits and carriers of a plan for a register of c.n qubits.
void plan_shape(SweepPlan &plan, const Circuit &c, int tile_qubits, int amp_bytes, bool reg_f64) {
    plan.n = c.n;
    plan.P = c.P;
    int m = tile_qubits > 0 ? tile_qubits : default_tile_qubits(c.n, amp_bytes, reg_f64);
    if (m > (reg_f64 ? 11 : 12)) m = reg_f64 ? 11 : 12;
    if (m > c.n) m = c.n;
    if (c.n - m > kMaxRest) fail(QNG_E_INVALID_ARG, "tile too small for this register (at most 24 qubits outside a tile)");
    plan.m = m;
    plan.rb = register_bits(m, amp_bytes);
    plan.carriers = c.n > m ? std::min(amp_bytes >= 16 ? 3 : 4, m - 1) : 0;
    if (c.n > m && m - plan.carriers < 2) fail(QNG_E_INVALID_ARG, "tile too small for the carrier qubits");
}

ColumnPlan plan_column(const Circuit &c, const SweepPlan &plan, int s, const std::vector<Event> &ev,
                       const SlotDest &sd) {
    ColumnPlan cp;
    cp.s = s;
    std::vector<uint8_t> done(ev.size(), 0);
    std::vector<int> pending(ev.size());
    for (size_t i = 0; i < ev.size(); ++i) pending[i] = (int)i;
    std::vector<uint8_t> tile;
    std::vector<int> emitted;
    while (!pending.empty()) {
        choose_and_emit(ev, done, pending, c.n, plan.m, plan.carriers, plan.width, tile, emitted);
        cp.passes.push_back(make_pass(c, sd, ev, emitted, tile, plan.rb, plan.carriers, plan.width));
    }
    return cp;
}

// Device images of all columns of a plan.
void flatten(SweepPlan &plan, const Circuit &c) {
    for (const ColumnPlan &cp : plan.cols) {
        plan.col_pass_begin.push_back((int64_t)plan.dev_passes.size());
        for (const HostPass &hp : cp.passes) {
            DevPass dp{};
            const uint32_t map_base = (uint32_t)plan.dev_maps.size();
            dp.op_begin = (uint32_t)plan.dev_ops.size();
            dp.n_ops = (uint32_t)hp.ops.size();
            dp.n_slots = (uint16_t)hp.slot_dest.size();
            dp.m = (uint8_t)hp.tile.size();
            dp.n = (uint8_t)c.n;
            dp.rb = (uint8_t)hp.rb;
            dp.map_load = map_base + (uint32_t)hp.map_load;
            for (size_t b = 0; b < hp.tile.size(); ++b) dp.tile_q[b] = hp.tile[b];
            std::vector<uint8_t> in(c.n, 0);
            for (uint8_t q : hp.tile) in[q] = 1;
            int k = 0;
            for (int q = 0; q < c.n; ++q)
                if (!in[q]) dp.rest_q[k++] = (uint8_t)q;
            dp.nrest = (uint8_t)k;
            bool has_cnot = false;
            for (DevOp op : hp.ops) {
                if (op.type == OP_ZSUM) dp.has_zsum = 1;
                if (op.type == OP_CNOT) has_cnot = true;
                if (op.type == OP_XPOSE) op.aux += (int32_t)map_base;
                op.type = device_opcode(op);
                const int h2 = device_handler2(op.type);
                if (h2 >= 0) {
                    op.hlo = op.hhi = 0;
                    op.h2 = 1u << h2;
                    plan.ctrl = true;
                } else {
                    const uint64_t hb = uint64_t(1) << device_handler(op.type);
                    op.hlo = (uint32_t)hb;
                    op.hhi = (uint32_t)(hb >> 32);
                    op.h2 = 0;
                }
                plan.dev_ops.push_back(op);
            }
            for (const DevMap &mp : hp.maps) plan.dev_maps.push_back(mp);
            plan.dev_passes.push_back(dp);
            plan.max_slots = std::max<int64_t>(plan.max_slots, dp.n_slots);
            plan.transposes += hp.transposes;
            if (has_cnot) ++plan.load_maps;
        }
    }
    plan.total_passes = (int64_t)plan.dev_passes.size();
    plan.total_ops = (int64_t)plan.dev_ops.size();
}

}  // namespace

// The forward plan of a metric plan: column k applies the gates at positions
// [from_k, rots[tops[k]].pos) to the forward register, from_0 = rots[0].pos and
// from_k = rots[tops[k-1]].pos, in tiles of the metric plan's width.  Its ops
// are the metric sweep's gate ops (OP_ROT, OP_DIAG, OP_CNOT, OP_CZ) ordered
// forward; given the shears of the gates themselves instead of their adjoints,
// the kernel applies the gates.
SweepPlan build_forward_plan(const Circuit &c, const std::vector<int> &tops, int tile_qubits, int amp_bytes,
                             bool reg_f64) {
    SweepPlan plan;
    plan.width = 0;
    plan_shape(plan, c, tile_qubits, amp_bytes, reg_f64);
    int from = c.rots[0].pos;
    for (int s : tops) {
        const int to = c.rots[s].pos;
        std::vector<Event> ev;
        for (int k = from; k < to; ++k) ev.push_back(unapply_event(c, k));
        plan.cols.push_back(plan_column(c, plan, s, ev, SlotDest{1, 0, 0}));
        from = to;
    }
    flatten(plan, c);
    return plan;
}

SweepPlan build_sweep_plan(const Circuit &c, int tile_qubits, int amp_bytes, int /*small*/, bool reg_f64,
                           int width, const std::vector<int> *rot_block) {
    if (width != 1 && width != 2 && width != 4) fail(QNG_E_INVALID_ARG, "column block width must be 1, 2 or 4");
    if (rot_block && width != 1) fail(QNG_E_INVALID_ARG, "a block-diagonal metric sweeps one column at a time");
    SweepPlan plan;
    plan.width = width;
    plan_shape(plan, c, tile_qubits, amp_bytes, reg_f64);
    // blocks from the top: columns P-1, P-1-width, ...; the lowest block may
    // have fewer real columns (its phi registers below column 1 stay unused)
    std::vector<int> tops;
    for (int s = c.P - 1; s >= 1; s -= width) tops.push_back(s);
    std::reverse(tops.begin(), tops.end());
    for (int s : tops)
        plan.cols.push_back(plan_column(c, plan, s, block_events(c, s, width, rot_block),
                                        SlotDest{c.P, s - width + 1, c.P * c.P}));
    flatten(plan, c);
    if (!c.controlled && !tops.empty())
        plan.forward = std::make_shared<SweepPlan>(build_forward_plan(c, tops, plan.m, amp_bytes, reg_f64));
    return plan;
}

SweepPlan build_gradient_plan(const Circuit &c, int tile_qubits, int amp_bytes, bool reg_f64) {
    SweepPlan plan;
    plan_shape(plan, c, tile_qubits, amp_bytes, reg_f64);
    if (c.P > 0) plan.cols.push_back(plan_column(c, plan, c.P, gradient_events(c), SlotDest{1, 0, 0}));
    flatten(plan, c);
    return plan;
}

size_t SweepPlan::device_bytes() const {
    return dev_passes.size() * sizeof(DevPass) + dev_ops.size() * sizeof(DevOp) + dev_maps.size() * sizeof(DevMap);
}

void SweepPlan::fill_info(qng_plan_info *out) const {
    out->passes = total_passes;
    out->elements = (int64_t)P * (P - 1) / 2;
    out->ops = total_ops;
    out->transposes = transposes;
    out->tile_qubits = m;
    out->small_n = n <= m ? 1 : 0;
}

uint8_t device_opcode(const DevOp &op) {
    const bool reg0 = op.b0 < kLocThread;
    const bool thr0 = op.b0 != kLocBase && !reg0;
    const int j = reg0 ? op.b0 : 0;
    if (reg0 && j > 3) fail(QNG_E_DEVICE, "device op: register position out of range (internal)");
    switch (op.type) {
    case OP_ROT:
    case OP_PRODROT:
    case OP_PROD: {
        if (!reg0) fail(QNG_E_DEVICE, "device op: X/Y operation off the registers (internal)");
        const int base = op.type == OP_ROT ? OPC_ROT_X : op.type == OP_PRODROT ? OPC_PRODROT_X : OPC_PROD_X;
        return (uint8_t)(base + (op.axis == 0 ? 0 : 4) + j);
    }
    case OP_PRODZ: return (uint8_t)(reg0 ? OPC_PRODZ_REG + j : thr0 ? OPC_PRODZ_THR : OPC_PRODZ_BASE);
    case OP_DIAG: return (uint8_t)(reg0 ? OPC_DIAG_REG + j : thr0 ? OPC_DIAG_THR : OPC_DIAG_BASE);
    case OP_PRODDIAG: return (uint8_t)(reg0 ? OPC_PRODDIAG_REG + j : thr0 ? OPC_PRODDIAG_THR : OPC_PRODDIAG_BASE);
    case OP_CNOT: {
        if (!reg0) fail(QNG_E_DEVICE, "device op: CNOT target off the registers (internal)");
        if (op.b1 < kLocThread) {
            if (op.b1 == op.b0 || op.b1 > 3) fail(QNG_E_DEVICE, "device op: bad CNOT control (internal)");
            return (uint8_t)(OPC_CNOT_REG + 4 * j + op.b1);
        }
        return (uint8_t)((op.b1 == kLocBase ? OPC_CNOT_BASE : OPC_CNOT_THR) + j);
    }
    case OP_CZ: return OPC_CZ;
    case OP_ZSUM: return OPC_ZSUM;
    case OP_XPOSE: return OPC_XPOSE;
    case OP_SEED: return OPC_SEED;
    case OP_CROT:
    case OP_PRODCROT:
    case OP_PRODC: {
        if (!reg0) fail(QNG_E_DEVICE, "device op: controlled X/Y operation off the registers (internal)");
        const int base = op.type == OP_CROT ? OPC_CROT_X : op.type == OP_PRODCROT ? OPC_PRODCROT_X : OPC_PRODC_X;
        return (uint8_t)(base + (op.axis == 0 ? 0 : 4) + j);
    }
    case OP_CDIAG: return OPC_CDIAG;
    case OP_PRODCDIAG: return OPC_PRODCDIAG;
    case OP_PRODCZ: return OPC_PRODCZ;
    case OP_CSEED: return OPC_CSEED;
    default: fail(QNG_E_DEVICE, "device op: unknown kind (internal)");
    }
    return 0;
}

int device_handler(uint8_t c) {
    if (c < OPC_ROT_Y) return HB_ROT_X + c;
    if (c < OPC_PRODROT_X) return HB_ROT_Y + (c - OPC_ROT_Y);
    if (c < OPC_PRODROT_Y) return HB_PRODROT_X + (c - OPC_PRODROT_X);
    if (c < OPC_PROD_X) return HB_PRODROT_Y + (c - OPC_PRODROT_Y);
    if (c < OPC_PROD_Y) return HB_PROD_X + (c - OPC_PROD_X);
    if (c < OPC_PRODZ_REG) return HB_PROD_Y + (c - OPC_PROD_Y);
    if (c < OPC_PRODZ_THR) return HB_PRODZ_REG + (c - OPC_PRODZ_REG);
    if (c <= OPC_PRODZ_BASE) return HB_PRODZ_UNI;
    if (c >= OPC_DIAG_REG && c < OPC_DIAG_THR) return HB_DIAG_REG + (c - OPC_DIAG_REG);
    if (c == OPC_DIAG_THR || c == OPC_DIAG_BASE) return HB_DIAG_UNI;
    if (c >= OPC_PRODDIAG_REG && c < OPC_PRODDIAG_THR) return HB_PRODDIAG_REG + (c - OPC_PRODDIAG_REG);
    if (c == OPC_PRODDIAG_THR || c == OPC_PRODDIAG_BASE) return HB_PRODDIAG_UNI;
    if (c >= OPC_CNOT_REG && c < OPC_CNOT_THR) {
        const int j = (c - OPC_CNOT_REG) / 4, k = (c - OPC_CNOT_REG) % 4;
        if (j == k) fail(QNG_E_DEVICE, "device handler: CNOT control on its target (internal)");
        return HB_CNOT_REG + 3 * j + (k < j ? k : k - 1);
    }
    if (c >= OPC_CNOT_THR && c < OPC_CNOT_BASE) return HB_CNOT_THR + (c - OPC_CNOT_THR);
    if (c >= OPC_CNOT_BASE && c < OPC_CZ) return HB_CNOT_BASE + (c - OPC_CNOT_BASE);
    if (c == OPC_CZ) return HB_CZ;
    if (c == OPC_ZSUM) return HB_ZSUM;
    if (c == OPC_XPOSE) return HB_XPOSE;
    if (c == OPC_SEED) return HB_SEED;
    fail(QNG_E_DEVICE, "device handler: unknown op code (internal)");
    return 0;
}

int device_handler2(uint8_t c) {
    // the controlled-rotation codes map onto the second word in order
    if (c < OPC_CROT_X) return -1;
    if (c > OPC_CSEED) fail(QNG_E_DEVICE, "device handler: unknown op code (internal)");
    static_assert(OPC_CSEED - OPC_CROT_X == HB2_CSEED && OPC_PRODC_Y - OPC_CROT_X == HB2_PRODC_Y &&
                      OPC_CDIAG - OPC_CROT_X == HB2_CDIAG,
                  "second handler word follows the op codes");
    return c - OPC_CROT_X;
}

void append_structure_key(const Circuit &c, std::vector<int32_t> &key) {
    key.push_back(c.n);
    key.push_back(c.M);
    key.push_back(c.P);
    for (const qng_gate &g : c.gates) {
        key.push_back(g.kind);
        key.push_back(g.q0);
        key.push_back(g.q1);
        key.push_back(g.param >= 0 ? 1 : 0);
    }
}

std::shared_ptr<const SweepPlan> SweepCache::get_shared(const Circuit &c, int tile_qubits, int amp_bytes, int small,
                                                        bool reg_f64, int width, const std::vector<int> *rot_block) {
    std::vector<int32_t> key = {tile_qubits, amp_bytes, small, reg_f64 ? 1 : 0, width};
    if (rot_block) {
        key.push_back(-2);
        key.insert(key.end(), rot_block->begin(), rot_block->end());
    }
    append_structure_key(c, key);
    auto it = plans.find(key);
    if (it != plans.end()) return it->second;
    if (plans.size() >= 256) plans.clear();
    auto p = std::make_shared<SweepPlan>(build_sweep_plan(c, tile_qubits, amp_bytes, small, reg_f64, width, rot_block));
    plans[key] = p;
    return p;
}

std::shared_ptr<const SweepPlan> SweepCache::get_gradient(const Circuit &c, int tile_qubits, int amp_bytes,
                                                          bool reg_f64) {
    std::vector<int32_t> key = {-1, tile_qubits, amp_bytes, reg_f64 ? 1 : 0};
    append_structure_key(c, key);
    auto it = plans.find(key);
    if (it != plans.end()) return it->second;
    if (plans.size() >= 256) plans.clear();
    auto p = std::make_shared<SweepPlan>(build_gradient_plan(c, tile_qubits, amp_bytes, reg_f64));
    plans[key] = p;
    return p;
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
    // keep the block registers within a quarter of the free memory
    while (B > 1 && (size_t)(1 + (plan.width + 1) * B) * state_bytes > free_bytes / 4) --B;
    fr.B = B;
    fr.partial_elems = (size_t)B * (size_t)plan.max_slots * (size_t)tiles + 16;
    return fr;
}

}  // namespace qng
