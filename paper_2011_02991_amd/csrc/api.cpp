// api.cpp -- the C ABI (include/qng.h): context, validation, workspace and the
// drivers of the recurrent metric, the reverse-sweep gradient and the step.
//
// Recurrence used by every driver (Sec. 2 recurrences and Sec. 3 Alg. 1,
// rewritten with the Pauli-generator form of the gate derivative, Sec. 2):
// for a rotation R_r = exp(i theta_r sigma_r / 2), dR_r/dtheta_r =
// (i/2) sigma_r R_r.  Let y_s be the state just before rotation s (all earlier
// gates applied) and V_{rs} the gates strictly between rotations r < s.  Then
//
//   L_rs = <d_r psi | d_s psi> = 1/4 <V^dag y_s | sigma_r | V^dag sigma_s y_s>,
//   T_s  = <psi | d_s psi>      = (i/2) <y_s | sigma_s | y_s>,   L_ss = 1/4.
//
// So column s starts from lambda = y_s, phi = sigma_s y_s (the paper's seed
// phi = dU_s psi_{s-1} after its first U_s^dag) and sweeps both registers
// backwards through the same adjoint gates; just before the adjoint of
// rotation r would be applied, <lambda|sigma_r|phi> is the paper's
// <mu|phi> = <dU_r lambda_{r-1} | phi> (mu := lambda; mu <- dU_r, never
// materialised since dU_r U_r^dag = (i/2) sigma_r).  psi advances by the gates
// between consecutive rotations (the paper's psi <- U_j).  O(P^2) gates, a
// constant number of state vectors.
//
// Energy gradient: d_r E = 2 Re <H psi | d_r psi>.  With lambda = H psi and
// phi = psi swept backwards from the last gate, d_r E = -Im <lambda|sigma_r|phi>
// at the same point of the sweep: O(P) gates, two registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "batch.hpp"
#include "circuit.hpp"
#include "fused.hpp"
#include "gram_kernels.hpp"
#include "kernels.hpp"
#include "noalloc.hpp"
#include "solve_kernels.hpp"
#include "sweep.hpp"

namespace qng {
void solve_shifted(int P, const double *G, double eps, const double *b, double *x);
}

using namespace qng;

// One register class of a batch: its schedule and, once captured, the hipGraph
// of its metric phase (valid for the workspace address it was captured with).
struct BatchClass {
    std::shared_ptr<BatchSchedule> sched;
    hipGraphExec_t graph = nullptr;
    const void *graph_ws = nullptr;
    std::vector<uint64_t> graph_ptrs;    // device addresses baked into the graph
    ~BatchClass() {
        if (graph) (void)hipGraphExecDestroy(graph);
    }
};

struct qng_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t mem_limit = 0;
    int opt_fusion = 1, opt_tile = 0, opt_streams = 0, opt_profile = 0, opt_small = 1, opt_f64_regs = 0;
    int opt_exact_products = 1;   // complex64: every inner-product term in FP64 (0: FP32 thread shares)
    int opt_graph = 1, opt_autotune = 0, opt_batch_tiles = 0, opt_block = 0, opt_metric_kind = 0;
    int opt_method = 0;   // 0: recurrence with O(1) states; 1: P derivative states and their Gram matrix
    int opt_state_chunk = 0;   // method 1: derivative states per chunk (0: automatic)
    std::vector<int> metric_blocks;   // block id per parameter (block-diagonal metric); empty = full
    std::string last_error;
    qng_stats stats{};
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // while set (the entry point that allocates nothing): the workspace is this
    // fixed device scratch instead of ws, and nothing is allocated
    char *fixed_ws = nullptr;
    size_t fixed_ws_bytes = 0;
    SweepCache sweep_cache;
    std::map<std::vector<int32_t>, std::shared_ptr<BatchClass>> batch_classes;
    std::map<std::vector<int32_t>, BatchTuning> tuned;
};

namespace {

thread_local std::string g_last_error;

#define HIPCHECK(call)                                                                                      \
    do {                                                                                                    \
        hipError_t _e = (call);                                                                             \
        if (_e != hipSuccess) fail(QNG_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(_e));       \
    } while (0)

template <typename F> qng_status guarded(qng_ctx *ctx, F &&f) {
    try {
        f();
        return QNG_OK;
    } catch (const Error &e) {
        if (ctx) ctx->last_error = e.msg;
        g_last_error = e.msg;
        return e.status;
    } catch (hipError_t e) {
        std::string m = std::string("HIP error: ") + hipGetErrorString(e);
        if (ctx) ctx->last_error = m;
        g_last_error = m;
        return QNG_E_DEVICE;
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->last_error = "host out of memory";
        g_last_error = "host out of memory";
        return QNG_E_OUT_OF_MEMORY;
    } catch (...) {
        if (ctx) ctx->last_error = "unknown error";
        g_last_error = "unknown error";
        return QNG_E_DEVICE;
    }
}

using Clock = std::chrono::steady_clock;
inline double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

constexpr int kMaxQubitsC128 = 32;
constexpr int kMaxQubitsC64 = 33;

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

DevMat2 dev(const Mat2 &m) {
    return DevMat2{m.a.real(), m.a.imag(), m.b.real(), m.b.imag(), m.c.real(), m.c.imag(), m.d.real(), m.d.imag()};
}

void check_in_state_host(int n, const double *in) {
    if (!in) return;
    const uint64_t dim = uint64_t(1) << n;
    double s = 0.0;
    for (uint64_t x = 0; x < 2 * dim; ++x) {
        if (!std::isfinite(in[x])) fail(QNG_E_NONFINITE, "input state is not finite");
        s += in[x] * in[x];
    }
    if (std::fabs(s - 1.0) > 1e-12) fail(QNG_E_NOT_NORMALIZED, "input state is not normalised (<in|in> - 1 = " +
                                                                   std::to_string(s - 1.0) + ")");
}

// -------------------------------------------------------------- workspace

struct Layout {
    size_t states = 0;      // offset of the state registers
    int n_states = 0;
    size_t state_bytes = 0;
    size_t staging = 0;     // complex128 copy of a host input state
    size_t partials = 0;    // reduction scratch
    size_t lraw = 0, traw = 0, graw = 0, eraw = 0, gout = 0, tout = 0, param_of = 0;
    size_t sweep = 0, sweep_bytes = 0;  // fused-sweep descriptors and partial sums
    size_t solve = 0;       // device solve of the step: A (NP*NP), y, x, grad (NP each), status
    size_t total = 0;
};

Layout plan_layout(int n, int P, size_t param_map_ints, size_t amp_bytes, int n_states, bool staging,
                   size_t sweep_bytes, int solve_params = -1) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    L.state_bytes = (size_t(1) << n) * amp_bytes;
    L.n_states = n_states;
    L.states = take(L.state_bytes * n_states);
    L.staging = staging ? take((size_t(1) << n) * 16) : 0;
    L.partials = take((size_t)reduce_blocks(n) * kStepMaxPhi * 16 + 16);
    L.lraw = take((size_t)P * P * 16 + (size_t)P * 16 + 16);
    L.traw = L.lraw + (size_t)P * P * 16;   // T right after L: column blocks reduce both into one array
    L.graw = take((size_t)P * 16 + 16);
    L.eraw = take(16);
    L.gout = take((size_t)P * P * 16 + 16);
    L.tout = take((size_t)P * 16 + 16);
    L.param_of = take(param_map_ints * 4 + 4);
    L.sweep_bytes = sweep_bytes;
    L.sweep = take(sweep_bytes + 16);
    if (solve_params >= 0) L.solve = take(((size_t)solve_params * solve_params + 3 * (size_t)solve_params) * 8 + 16);
    L.total = off;
    return L;
}

char *ensure_workspace(qng_ctx *ctx, size_t bytes) {
    if (ctx->fixed_ws) {
        if (bytes > ctx->fixed_ws_bytes)
            fail(QNG_E_OUT_OF_MEMORY, "this call needs " + std::to_string(bytes) +
                                          " bytes of device scratch; the fixed scratch of the entry point that "
                                          "allocates nothing holds " + std::to_string(ctx->fixed_ws_bytes));
        return ctx->fixed_ws;
    }
    if (ctx->mem_limit && bytes > ctx->mem_limit)
        fail(QNG_E_OUT_OF_MEMORY, "workspace of " + std::to_string(bytes) + " bytes exceeds the context limit of " +
                                      std::to_string(ctx->mem_limit));
    if (bytes <= ctx->ws_bytes) return (char *)ctx->ws;
    if (ctx->ws) {
        HIPCHECK(hipStreamSynchronize(ctx->stream));
        HIPCHECK(hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    size_t free_b = 0, total_b = 0;
    HIPCHECK(hipMemGetInfo(&free_b, &total_b));
    if (bytes > free_b)
        fail(QNG_E_OUT_OF_MEMORY, "workspace of " + std::to_string(bytes) + " bytes exceeds free device memory (" +
                                      std::to_string(free_b) + ")");
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(QNG_E_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    ctx->ws = p;
    ctx->ws_bytes = bytes;
    return (char *)p;
}

// -------------------------------------------------------------- the engine

struct Problem {
    Circuit circ;
    std::vector<Mat2> fwd, adj;       // per gate position (rotations only)
    std::vector<int> param_of;        // rotation (list order) -> parameter index
    // device image of the parameter map: param_of [P], then the rotations of
    // each parameter as off [NP + 1] and rot [P] (rot[off[a] .. off[a+1]) carry
    // a), then the block of each rotation [P] (block-diagonal metric), then
    // the control qubit of each rotation [P] (-1: plain rotation)
    std::vector<int> param_map;
    std::vector<PauliTerm> ham;
    bool has_ham = false;
    std::vector<int> rot_block;       // block id per rotation; empty = full metric
    bool l_only = false;              // metric without the conj(T_i) T_j term
};

// ints of a Problem's parameter map image
inline size_t param_map_ints(const Circuit &c) { return (size_t)4 * c.P + c.NP + 1; }
inline size_t rot_ctrl_offset(const Circuit &c) { return (size_t)3 * c.P + c.NP + 1; }

// lower: rewrite Pauli-string rotations as fixed rotations, CNOTs and an RZ
// (lower_strings) so that the fused passes take the circuit; asked for by the
// entry points that sweep when fusion is on.
Problem make_problem(const qng_circuit *c, const double *theta, const qng_pauli_sum *h, bool lower = false) {
    Problem p;
    p.circ = compile_circuit(c);
    if (lower && p.circ.has_strings && strings_lowerable(p.circ)) p.circ = lower_strings(p.circ);
    p.fwd.resize(p.circ.M);
    p.adj.resize(p.circ.M);
    for (const Rot &r : p.circ.rots) {
        p.fwd[r.pos] = rotation(r.axis, theta[r.param]);
        p.adj[r.pos] = adjoint(p.fwd[r.pos]);
        p.param_of.push_back(r.param);
    }
    for (int pos = 0; pos < p.circ.M; ++pos)
        if (p.circ.is_fixed_rotation(pos)) {
            const int kind = p.circ.gates[pos].kind;
            p.fwd[pos] = rotation(kind == QNG_RX ? AX_X : kind == QNG_RY ? AX_Y : AX_Z, p.circ.fixed_angle[pos]);
            p.adj[pos] = adjoint(p.fwd[pos]);
        }
    const int P = p.circ.P, NP = p.circ.NP;
    p.param_map = p.param_of;
    std::vector<int> count(NP + 1, 0);
    for (int r = 0; r < P; ++r) ++count[p.param_of[r] + 1];
    for (int a = 0; a < NP; ++a) count[a + 1] += count[a];
    p.param_map.insert(p.param_map.end(), count.begin(), count.end());
    std::vector<int> rot(P), fill(count.begin(), count.end() - 1);
    for (int r = 0; r < P; ++r) rot[fill[p.param_of[r]]++] = r;
    p.param_map.insert(p.param_map.end(), rot.begin(), rot.end());
    p.param_map.resize(rot_ctrl_offset(p.circ), 0);   // rotation blocks: set by apply_metric_settings
    for (const Rot &r : p.circ.rots) p.param_map.push_back(r.ctrl);
    if (h) {
        p.ham = compile_hamiltonian(c, h);
        p.has_ham = true;
    }
    return p;
}

// Arithmetic of the fused sweep passes for a storage precision (amp bytes per
// amplitude): FP64 for complex128 or when FP64 registers are asked for, else
// FP32 registers with FP32 thread shares of the products or, on request,
// every product in FP64.
int sweep_reg_mode(const qng_ctx *ctx, size_t amp) {
    if (amp == 16 || ctx->opt_f64_regs) return REG_F64;
    return ctx->opt_exact_products ? REG_F32_EXACT : REG_F32;
}

// The context's metric settings for a problem: block-diagonal blocks (when the
// circuit has the number of parameters they were given for) and the L-only
// form.
void apply_metric_settings(const qng_ctx *ctx, Problem &p) {
    const Circuit &c = p.circ;
    p.l_only = ctx->opt_metric_kind == 1;
    if (!ctx->metric_blocks.empty()) {
        if ((int)ctx->metric_blocks.size() != c.NP)
            fail(QNG_E_INVALID_ARG, "metric blocks were set for " + std::to_string(ctx->metric_blocks.size()) +
                                        " parameters, the circuit has " + std::to_string(c.NP));
        p.rot_block.resize(c.P);
        for (int r = 0; r < c.P; ++r) p.rot_block[r] = ctx->metric_blocks[p.param_of[r]];
        std::copy(p.rot_block.begin(), p.rot_block.end(), p.param_map.begin() + 2 * c.P + c.NP + 1);
    }
}

// Gate `pos` of a problem (or its adjoint) on one register or two.  A
// Pauli-string rotation's fwd/adj hold cos(theta/2) on the diagonal and
// +-i sin(theta/2) off it (the RX matrix of its angle), i.e. c + (i s) S.
template <typename R>
void apply_gate(const Problem &pb, int pos, bool adjoint_gate, void *s0, void *s1, hipStream_t st) {
    const qng_gate &g = pb.circ.gates[pos];
    const int n = pb.circ.n;
    const Mat2 &mm = adjoint_gate ? pb.adj[pos] : pb.fwd[pos];
    if (g.kind == QNG_CNOT) launch_cnot<R>(s0, s1, n, g.q0, g.q1, st);
    else if (g.kind == QNG_CZ) launch_cz<R>(s0, s1, n, g.q0, g.q1, st);
    else if (g.kind == QNG_RPAULI) {
        const Rot &r = pb.circ.rots[pb.circ.rot_at[pos]];
        launch_apply_string<R>(s0, s1, n, r.flip, r.zy, r.n_y, mm.a.real(), mm.b.real(), mm.b.imag(), st);
    } else if (g.kind >= QNG_CRX) launch_apply_c1q<R>(s0, s1, n, g.q0, g.q1, dev(mm), st);
    else launch_apply_1q<R>(s0, s1, n, g.q0, dev(mm), st);
}

template <typename R> struct Engine {
    qng_ctx *ctx;
    const Problem &pb;
    hipStream_t st;
    int n;
    void *regs[3];            // psi, lambda, phi
    size_t state_bytes;
    double *partials_, *lraw_, *traw_, *graw_, *eraw_;

    Engine(qng_ctx *c, const Problem &p, hipStream_t s, void *psi, void *lam, void *phi, size_t sb, double *part,
           double *lraw, double *traw, double *graw, double *eraw)
        : ctx(c), pb(p), st(s), n(p.circ.n), regs{psi, lam, phi}, state_bytes(sb), partials_(part), lraw_(lraw),
          traw_(traw), graw_(graw), eraw_(eraw) {}

    // fused reverse sweep of the gradient (nullptr: one kernel per primitive)
    const SweepPlan *gplan = nullptr;
    char *gscratch = nullptr;
    size_t gscratch_bytes = 0;
    int reg_mode = REG_F32;
    bool stepped = false;     // one kernel per sweep step (circuits the fused passes do not take)

    // registers 0..2 as given; further ones (the phi registers of a stepped
    // block) follow psi contiguously, as run() lays them out
    void *state(int k) const { return k < 3 ? regs[k] : (char *)regs[0] + (size_t)k * state_bytes; }
    double *partials() const { return partials_; }
    double *lraw() const { return lraw_; }
    double *traw() const { return traw_; }
    double *graw() const { return graw_; }
    double *eraw() const { return eraw_; }

    void apply(int pos, bool adjoint_gate, void *s0, void *s1) {
        ++ctx->stats.other_launches;
        apply_gate<R>(pb, pos, adjoint_gate, s0, s1, st);
    }

    // <a| K |b> with K = sigma_q, or |1><1|_ctrl (x) sigma_q for ctrl >= 0
    void prod(const void *a, const void *b, int q, int axis, double *dest, int ctrl = -1) {
        ctx->stats.other_launches += 2;
        launch_pauli_prod<R>(a, b, n, q, axis, partials(), dest, st, ctrl);
    }

    // One back-sweep step of rotation r (gate position pos) over lambda and the
    // phi registers of sr: <lambda|K_r|phi_k> into dests (if given), then the
    // adjoint of r on all of them.
    StepGate step_gate(const Rot &r, int pos) const {
        StepGate g{};
        g.n = n;
        const Mat2 &a = pb.adj[pos];
        if (r.string >= 0) {
            // adjoint c - i s S = c + kappa S' with kappa = (-i s) w (a.b holds -i s)
            g.kind = STEP_STRING;
            g.flip = r.flip;
            g.zy = r.zy;
            cd w(1, 0);
            for (int k = 0; k < (r.n_y & 3); ++k) w *= cd(0, -1);
            g.wr = w.real();
            g.wi = w.imag();
            const cd kappa = a.b * w;
            g.m[0] = a.a.real();
            g.m[2] = kappa.real();
            g.m[3] = kappa.imag();
        } else {
            g.kind = r.ctrl >= 0 ? STEP_C1Q : STEP_1Q;
            g.q = r.qubit;
            g.c = r.ctrl;
            g.axis = r.axis;
            const cd e[4] = {a.a, a.b, a.c, a.d};
            for (int k = 0; k < 4; ++k) {
                g.m[2 * k] = e[k].real();
                g.m[2 * k + 1] = e[k].imag();
            }
        }
        return g;
    }
    void step(const StepRegs &sr, int r, int pos, const StepDests *dests) {
        ctx->stats.other_launches += dests && sr.n_phi ? 2 : 1;
        launch_sweep_step<R>(sr, step_gate(pb.circ.rots[r], pos), partials(), dests, st);
    }

    // <a| K_r |b> for the generator K_r of rotation r
    void rprod(const void *a, const void *b, const Rot &r, double *dest) {
        if (r.string < 0) return prod(a, b, r.qubit, r.axis, dest, r.ctrl);
        ctx->stats.other_launches += 2;
        launch_string_prod<R>(a, b, n, r.flip, r.zy, r.n_y, partials(), dest, st);
    }

    // lam = y, phi = K_r y
    void rseed(const void *y, void *lam, void *phi, const Rot &r) {
        ++ctx->stats.other_launches;
        if (r.string < 0) launch_seed<R>(y, lam, phi, n, r.qubit, r.axis, st, r.ctrl);
        else launch_seed_string<R>(y, lam, phi, n, r.flip, r.zy, r.n_y, st);
    }

    // psi (state 0) <- |in>.  in_c128: device complex128 or nullptr.
    void init(const void *in_c128) {
        ++ctx->stats.other_launches;
        launch_init_state<R>(state(0), n, in_c128, st);
    }

    // Recurrent metric, one kernel per primitive.  On return psi holds y_{P-1}
    // (the state just before the last rotation) and `pos` its gate position.
    int metric_unfused() {
        const Circuit &c = pb.circ;
        void *psi = state(0), *lam = state(1), *phi = state(2);
        int pos = 0;
        const int p0 = c.P ? c.rots[0].pos : 0;
        for (int s = 0; s < c.P; ++s) {
            const Rot &rs = c.rots[s];
            for (; pos < rs.pos; ++pos) apply(pos, false, psi, nullptr);   // psi <- gates up to rotation s
            rprod(psi, psi, rs, traw() + 2 * s);                             // <y_s|K_s|y_s>
            // controlled rotation: <y_s|K_s^2|y_s> = Prob(control = 1) on the diagonal (Sec. 2)
            if (rs.ctrl >= 0) prod(psi, psi, rs.ctrl, -1, lraw() + 2 * ((size_t)s * c.P + s), rs.ctrl);
            if (s == 0) continue;
            // block-diagonal metric: the column stops at the lowest rotation of its block
            int lo = 0;
            if (!pb.rot_block.empty()) {
                lo = -1;
                for (int r = s - 1; r >= 0; --r)
                    if (pb.rot_block[r] == pb.rot_block[s]) lo = r;
                if (lo < 0) continue;
            }
            const int plo = lo ? c.rots[lo].pos : p0;
            rseed(psi, lam, phi, rs);
            for (int k = rs.pos - 1; k >= plo; --k) {
                const int r = c.rot_at[k];
                if (r >= 0) {
                    const Rot &rr = c.rots[r];
                    if (pb.rot_block.empty() || pb.rot_block[r] == pb.rot_block[s]) {
                        rprod(lam, phi, rr, lraw() + 2 * ((size_t)r * c.P + s));
                        ++ctx->stats.elements;
                    }
                    if (k > plo) apply(k, true, lam, phi);
                } else {
                    apply(k, true, lam, phi);
                }
            }
        }
        return pos;
    }

    // Recurrent metric for circuits the fused passes do not take (Pauli-string
    // rotations): columns in blocks of up to `width`
    // consecutive rotations share one lambda sweep, as in the fused passes --
    // lambda swept back from the top column is the forward state y_r at every
    // rotation r, so the block's lower columns are seeded from it on the way
    // down -- and every step is one kernel over lambda and the block's phi
    // registers (state(2) .. state(1 + width)).  On return psi holds y_{P-1}.
    int metric_stepped(int width) {
        const Circuit &c = pb.circ;
        void *psi = state(0), *lam = state(1);
        int pos = 0;
        const int p0 = c.P ? c.rots[0].pos : 0;
        for (int s0 = 0; s0 < c.P; s0 += width) {
            const int s1 = std::min(c.P, s0 + width) - 1;
            for (int s = s0; s <= s1; ++s) {
                const Rot &rs = c.rots[s];
                for (; pos < rs.pos; ++pos) apply(pos, false, psi, nullptr);
                rprod(psi, psi, rs, traw() + 2 * s);                      // <y_s|K_s|y_s>
                if (rs.ctrl >= 0) prod(psi, psi, rs.ctrl, -1, lraw() + 2 * ((size_t)s * c.P + s), rs.ctrl);
            }
            if (s1 == 0) continue;
            StepRegs sr{};
            sr.lam = lam;
            int col[kStepMaxPhi];
            rseed(psi, lam, state(2), c.rots[s1]);
            sr.phi[0] = state(2);
            col[0] = s1;
            sr.n_phi = 1;
            for (int k = c.rots[s1].pos - 1; k >= p0; --k) {
                const int r = c.rot_at[k];
                if (r < 0) {
                    const qng_gate &g = c.gates[k];
                    ++ctx->stats.other_launches;
                    launch_fixed_multi<R>(sr, n, g.kind == QNG_CNOT, g.q0, g.q1, st);
                    continue;
                }
                StepDests d{};
                d.base = lraw();
                for (int j = 0; j < sr.n_phi; ++j) d.off[j] = (int64_t)r * c.P + col[j];
                step(sr, r, k, &d);
                ctx->stats.elements += sr.n_phi;
                if (r >= s0 && r > 0) {           // lambda = y_r: column r starts here
                    rseed(lam, lam, state(2 + sr.n_phi), c.rots[r]);
                    sr.phi[sr.n_phi] = state(2 + sr.n_phi);
                    col[sr.n_phi++] = r;
                }
            }
        }
        return pos;
    }

    // From psi at gate position pos: finish the forward pass, lambda = H psi,
    // E = <psi|lambda>, then the reverse sweep for the gradient (the fused
    // passes of the gradient plan when one is set, one kernel per sweep step for
    // Pauli-string rotations left as they are, else one kernel per primitive).  psi_copy_c128
    // (nullable) receives the final state before the sweep modifies psi.
    void finish_energy_grad(int pos, bool want_grad, void *psi_copy_c128) {
        const Circuit &c = pb.circ;
        void *psi = state(0), *lam = state(1);
        for (; pos < c.M; ++pos) apply(pos, false, psi, nullptr);
        if (psi_copy_c128) { ++ctx->stats.other_launches; launch_to_c128<R>(psi, psi_copy_c128, n, st); }
        energy(psi, lam);
        if (!want_grad || c.P == 0) return;
        if (gplan) {
            run_fused_gradient<R>(*gplan, c, pb.adj, lam, psi, graw(), gscratch, gscratch_bytes, st, &ctx->stats,
                                  ctx->opt_profile != 0, reg_mode);
            return;
        }
        const int p0 = c.rots[0].pos;
        if (stepped) {
            // one kernel per rotation: <lambda|K_r|psi> and the adjoint on both
            StepRegs sr{};
            sr.lam = lam;
            sr.phi[0] = psi;
            sr.n_phi = 1;
            for (int k = c.M - 1; k >= p0; --k) {
                const int r = c.rot_at[k];
                if (r >= 0) {
                    StepDests d{};
                    d.base = graw();
                    d.off[0] = r;
                    step(sr, r, k, &d);
                } else {
                    apply(k, true, lam, psi);
                }
            }
            return;
        }
        for (int k = c.M - 1; k >= p0; --k) {
            const int r = c.rot_at[k];
            if (r >= 0) {
                const Rot &rr = c.rots[r];
                rprod(lam, psi, rr, graw() + 2 * r);
                if (k > p0) apply(k, true, lam, psi);
            } else {
                apply(k, true, lam, psi);
            }
        }
    }

    // out = H psi and E = <psi|out> (into eraw), one pass over the register per
    // chunk of terms
    void energy(const void *psi, void *out) {
        std::vector<HamTerm> terms(pb.ham.size());
        for (size_t t = 0; t < pb.ham.size(); ++t) {
            const PauliTerm &h = pb.ham[t];
            cd c(h.coeff, 0.0);
            for (int k = 0; k < (h.n_y & 3); ++k) c *= cd(0, -1);
            terms[t] = HamTerm{h.flip, h.zy, c.real(), c.imag()};
        }
        ctx->stats.other_launches += 1 + (int64_t)(terms.size() + kHamChunk - 1) / kHamChunk;
        launch_pauli_sum<R>(psi, out, n, terms.data(), (int)terms.size(), partials(), eraw(), st);
    }
};

struct CallSpec {
    bool metric = false, grad = false;
    const double *in_host = nullptr;      // complex128 host input (nullable)
    const void *in_dev = nullptr;         // complex128 device input (nullable)
    void *psi_out_dev = nullptr;          // complex128 device copy of the final state (nullable)
    bool host_call = false;               // synchronous host-pointer entry point: time each phase
    const void *psi_final_dev = nullptr;  // gradient from a given final state (nullable)
    bool real_products = false;           // fused metric: real parts of L only (the caller needs Re G)
    bool device_solve = false;            // reserve the workspace of the step's device solve
};

// Columns per lambda sweep of the fused metric.  Blocks of two columns need
// full tiles of at least 11 qubits (8 or 16 amplitudes per thread); option
// value 0 picks the default.
// Columns per lambda sweep (QNG_OPT_BLOCK_COLUMNS, 0 = automatic): four for
// FP32 registers in tiles of 11 qubits (8 amplitudes per thread; measured at
// n = 26, complex64: 7 % less sweep time than two columns in tiles of 12)
// without controlled rotations; else two for full tiles of 8 or 16
// amplitudes per thread; else one.
int block_width(int opt_block, const Circuit &c, int opt_tile, int amp, bool f64, int max_width = kMaxBlockWidth) {
    int m = opt_tile > 0 ? opt_tile : default_tile_qubits(c.n, amp, f64);
    if (m > (f64 ? 11 : 12)) m = f64 ? 11 : 12;
    if (m > c.n) m = c.n;
    const bool four = !f64 && !c.controlled && (opt_tile == 0 || opt_tile == 11) && c.n >= 11;
    const int want = std::min(opt_block > 0 ? opt_block : (four ? 4 : kDefaultBlockWidth), max_width);
    if (want == 4 && four) return 4;
    return (want >= 2 && register_bits(m, amp) >= 3 && m - register_bits(m, amp) == 8) ? 2 : 1;
}

// Smallest register for which the batched step picks four-column blocks by itself.
constexpr int kBatchFourMinQubits = 18;

// Tile width a plan of `width` columns per sweep is built for: four-column
// blocks take tiles of 11 qubits (8 amplitudes per thread in FP32 registers).
int plan_tile(int width, int opt_tile) { return width == 4 && opt_tile == 0 ? 11 : opt_tile; }

// G and T in parameter order from the raw L and T of the rotations: with one
// parameter per rotation, unpacked straight into gout/tout; with shared
// parameters, unpacked in rotation order into gout/tout and contracted
// (J^T G J, J^T T) into `spare`, which must hold NP*NP + NP complex (the raw L
// of P*P >= that is dead by then).  G and T are set to where the results are.
void unpack_to_params(const Problem &pb, const double *lraw, const double *traw, const int *param_map_dev,
                      double *gout, double *tout, double *spare, double *&G, double *&T, hipStream_t st) {
    const Circuit &c = pb.circ;
    const int *rot_block = pb.rot_block.empty() ? nullptr : param_map_dev + 2 * c.P + c.NP + 1;
    const int *rot_ctrl = c.controlled ? param_map_dev + rot_ctrl_offset(c) : nullptr;
    if (!c.shared) {
        launch_unpack_metric(lraw, traw, param_map_dev, c.P, gout, tout, rot_block, rot_ctrl, pb.l_only, st);
        G = gout;
        T = tout;
        return;
    }
    launch_unpack_metric(lraw, traw, nullptr, c.P, gout, tout, rot_block, rot_ctrl, pb.l_only, st);
    G = spare;
    T = spare + 2 * (size_t)c.NP * c.NP;
    launch_contract_metric(gout, tout, c.P, param_map_dev + c.P, param_map_dev + c.P + c.NP + 1, c.NP, G, T, st);
}

struct CallResult {
    // device pointers into the workspace
    double *G = nullptr, *T = nullptr, *graw = nullptr, *eraw = nullptr;
    const int *param_of = nullptr;
    char *solve = nullptr;                // CallSpec::device_solve: the solve's workspace
};

template <typename R>
CallResult run(qng_ctx *ctx, const Problem &pb, const CallSpec &spec) {
    const Circuit &c = pb.circ;
    const int n = c.n;
    const size_t amp = 2 * sizeof(R);
    const size_t V = (size_t(1) << n) * amp;
    // the fused passes take single-qubit and controlled rotations, CNOT and CZ;
    // Pauli-string rotations run one kernel per sweep step
    const bool fused = ctx->opt_fusion != 0 && spec.metric && c.P > 1 && !c.has_strings;
    // derivative-state variant: every column's swept phi register is kept and
    // the metric is their Gram matrix (P + 1 more states)
    const bool states = ctx->opt_method == 1 && spec.metric && c.P > 1;
    if (states && (!fused || !pb.rot_block.empty()))
        fail(QNG_E_UNSUPPORTED, "the derivative-state variant takes the fused passes (no Pauli string without a "
                                "letter) and the full metric");
    const SweepPlan *plan = nullptr;
    FusedRun fr;
    size_t scratch = 0, gram_bytes = 0;
    int chunk_cols = 0;
    int n_states = spec.metric ? 4 : 2;   // the gradient alone needs psi and lambda = H psi
    int n_block_states = 0;
    if (fused) {
        const bool f64_regs = amp == 16 || ctx->opt_f64_regs;
        const bool blocked = !pb.rot_block.empty();
        const int width = blocked ? 1 : block_width(ctx->opt_block, c, ctx->opt_tile, (int)amp, f64_regs);
        plan = &ctx->sweep_cache.get(c, plan_tile(width, ctx->opt_tile), (int)amp, ctx->opt_small, f64_regs, width,
                                     blocked ? &pb.rot_block : nullptr);
        size_t free_b = 0, total_b = 0;
        HIPCHECK(hipMemGetInfo(&free_b, &total_b));
        const size_t avail = free_b + ctx->ws_bytes;
        const size_t cap = ctx->mem_limit ? std::min(avail, ctx->mem_limit) : avail;
        // the derivative-state variant: chunk_cols columns per chunk (all P - 1
        // columns above column 0 when they fit), kept after the block registers
        auto configure = [&](int cols) {
            const size_t kept = states ? kept_states(c.P, cols) * V : 0;
            fr = fused_config(*plan, ctx->opt_streams, V, cap > kept ? cap - kept : 0);
            gram_bytes = states ? states_gram_bytes(n, c.P, cols) : 0;
            scratch = fused_scratch_bytes(*plan, fr, c.M) + gram_bytes;
            n_block_states = std::max(4, 1 + (plan->width + 1) * fr.B);
            n_states = n_block_states + (states ? (int)kept_states(c.P, cols) : 0);
            return plan_layout(n, c.P, param_map_ints(c), amp, n_states, spec.in_host != nullptr, scratch,
                               spec.device_solve ? c.NP : -1).total;
        };
        if (states) {
            const int all = c.P - 1;
            // (a chunk holds whole column blocks: at least one)
            chunk_cols = ctx->opt_state_chunk > 0 ? std::min(std::max(ctx->opt_state_chunk, plan->width), all) : all;
            if (ctx->opt_state_chunk == 0) {
                // the most columns per chunk that fit (two chunks held at once below all)
                while (chunk_cols >= plan->width && configure(chunk_cols) > cap)
                    chunk_cols = chunk_cols == all ? all / 2 : chunk_cols - 1;
                if (chunk_cols < plan->width)
                    fail(QNG_E_OUT_OF_MEMORY, "the derivative-state variant needs at least " +
                                                  std::to_string(kept_states(c.P, plan->width)) + " states of " +
                                                  std::to_string(V) + " bytes (chunks of one column block); " +
                                                  std::to_string(cap) + " bytes are available");
            }
        }
        configure(chunk_cols);
        ctx->stats.block_columns = plan->width;
    }
    std::shared_ptr<const SweepPlan> gplan;
    const bool f64_regs = amp == 16 || ctx->opt_f64_regs;
    if (ctx->opt_fusion != 0 && spec.grad && c.P > 0 && !c.has_strings) {
        gplan = ctx->sweep_cache.get_gradient(c, ctx->opt_tile, (int)amp, f64_regs);
        scratch = std::max(scratch, fused_gradient_scratch_bytes(*gplan, c.M));
    }
    // circuits the fused passes do not take: one kernel per sweep step, with up
    // to kStepMaxPhi columns per lambda sweep as memory allows (half of what is
    // free, and the context's limit)
    const bool stepped = ctx->opt_fusion != 0 && c.has_strings;
    int step_width = 0;
    if (stepped && spec.metric && pb.rot_block.empty() && c.P > 1) {
        size_t free_b = 0, total_b = 0;
        HIPCHECK(hipMemGetInfo(&free_b, &total_b));
        size_t budget = (free_b + ctx->ws_bytes) / 2;
        if (ctx->mem_limit) budget = std::min(budget, ctx->mem_limit);
        const size_t fixed = (size_t)c.P * c.P * 48 + ((size_t)1 << n) * 16 + ((size_t)64 << 20);
        const size_t fit = budget > fixed ? (budget - fixed) / V : 0;
        step_width = (int)std::min<size_t>(kStepMaxPhi, fit > 2 ? fit - 2 : 0);
        if (step_width < 2) step_width = 0;     // the one-column loop needs 3 registers
        n_states = std::max(n_states, 2 + step_width);
    }
    Layout L = plan_layout(n, c.P, param_map_ints(c), amp, n_states, spec.in_host != nullptr, scratch,
                           spec.device_solve ? c.NP : -1);
    char *base = ensure_workspace(ctx, L.total);
    hipStream_t st = ctx->stream;
    char *sb = base + L.states;
    Engine<R> e(ctx, pb, st, sb, sb + L.state_bytes, sb + 2 * L.state_bytes, L.state_bytes,
                (double *)(base + L.partials), (double *)(base + L.lraw), (double *)(base + L.traw),
                (double *)(base + L.graw), (double *)(base + L.eraw));
    if (gplan) {
        e.gplan = gplan.get();
        e.gscratch = base + L.sweep;
        e.gscratch_bytes = L.sweep_bytes;
        e.reg_mode = sweep_reg_mode(ctx, amp);
    }
    e.stepped = stepped;

    const void *in_c128 = spec.in_dev;
    if (spec.in_host) {
        HIPCHECK(hipMemcpyAsync(base + L.staging, spec.in_host, (size_t(1) << n) * 16, hipMemcpyHostToDevice, st));
        in_c128 = base + L.staging;
    }
    if (c.P)
        HIPCHECK(hipMemcpyAsync(base + L.param_of, pb.param_map.data(), pb.param_map.size() * 4, hipMemcpyHostToDevice,
                                st));
    CallResult res;
    res.graw = e.graw();
    res.param_of = (const int *)(base + L.param_of);
    res.eraw = e.eraw();
    if (spec.device_solve) res.solve = base + L.solve;
    int pos = 0;
    if (spec.metric) {
        auto t0 = Clock::now();
        e.init(in_c128);
        // raw L and T (T right after L); the derivative-state variant without
        // the complex G writes the real parts of T alone
        if (c.P) HIPCHECK(hipMemsetAsync(e.lraw(), 0, ((size_t)c.P * c.P + c.P) * 16, st));
        if (fused) {
            FusedBuffers fb;
            fb.states = base + L.states;
            fb.state_bytes = L.state_bytes;
            fb.scratch = base + L.sweep;
            fb.scratch_bytes = L.sweep_bytes;
            fb.traw = e.traw();
            fb.lraw = e.lraw();
            fb.reduce_partials = e.partials();
            if (states) {
                fb.scratch_bytes = L.sweep_bytes - gram_bytes;
                fb.gram_partials = (double *)(base + L.sweep + fb.scratch_bytes);
                fb.gram_signs = (int8_t *)(base + L.sweep + L.sweep_bytes) - align256((size_t)c.P + 1 + 64);
                fb.dummy = base + L.states + (size_t)n_block_states * L.state_bytes;
                fb.xi = fb.dummy + L.state_bytes;
                pos = run_states_metric<R>(*plan, fr, c, pb.fwd, pb.adj, fb, chunk_cols, [&] { e.init(in_c128); }, st,
                                           &ctx->stats, ctx->opt_profile != 0, spec.real_products);
            } else {
                pos = run_fused_metric<R>(*plan, fr, c, pb.fwd, pb.adj, fb, st, &ctx->stats, ctx->opt_profile != 0,
                                          sweep_reg_mode(ctx, amp), spec.real_products);
            }
        } else if (step_width > 0) {
            pos = e.metric_stepped(step_width);
        } else {
            pos = e.metric_unfused();
        }
        unpack_to_params(pb, e.lraw(), e.traw(), (const int *)(base + L.param_of), (double *)(base + L.gout),
                         (double *)(base + L.tout), e.lraw(), res.G, res.T, st);
        if (spec.host_call || ctx->opt_profile) HIPCHECK(hipStreamSynchronize(st));
        ctx->stats.metric_ms = ms_since(t0);
    }
    if (spec.grad) {
        auto t0 = Clock::now();
        if (spec.psi_final_dev) {
            launch_init_state<R>(e.state(0), n, spec.psi_final_dev, st);
            pos = c.M;
        } else if (!spec.metric) {
            e.init(in_c128);
            pos = 0;
        }
        e.finish_energy_grad(pos, true, spec.psi_out_dev);
        if (spec.host_call || ctx->opt_profile) HIPCHECK(hipStreamSynchronize(st));
        ctx->stats.grad_ms = ms_since(t0);
    } else if (spec.psi_out_dev) {
        // energy only
        if (!spec.metric) {
            e.init(in_c128);
            pos = 0;
        }
        e.finish_energy_grad(pos, false, spec.psi_out_dev);
    }
    return res;
}

void reset_stats(qng_ctx *ctx) { ctx->stats = qng_stats{}; }

void require_ctx(qng_ctx *ctx) {
    if (!ctx) fail(QNG_E_INVALID_ARG, "context is NULL");
    HIPCHECK(hipSetDevice(ctx->device));
}

int max_qubits(qng_precision prec) { return prec == QNG_C64 ? kMaxQubitsC64 : kMaxQubitsC128; }

void check_prec(int prec) {
    if (prec != QNG_C128 && prec != QNG_C64) fail(QNG_E_INVALID_ARG, "unknown precision");
}

template <typename F> void dispatch(qng_precision prec, F &&f) {
    if (prec == QNG_C64) f((float)0);
    else f((double)0);
}

// d E / d theta_a = sum over the rotations r carrying a of -Im graw[r]
void host_unpack_grad(const std::vector<double> &graw, const Problem &pb, double *grad) {
    for (int a = 0; a < pb.circ.NP; ++a) grad[a] = 0.0;
    for (size_t r = 0; r < pb.param_of.size(); ++r) grad[pb.param_of[r]] -= graw[2 * r + 1];
}

// The gradient in parameter order on the device, from the raw per-rotation
// products of a run: -Im graw[r] into its parameter (summed over the rotations
// of a shared parameter).
void device_grad(const CallResult &r, const Problem &pb, double *grad, hipStream_t st) {
    const int P = pb.circ.P;
    if (!P) return;
    if (!pb.circ.shared) launch_grad_from_raw(r.graw, r.param_of, P, grad, st);
    else launch_grad_contract(r.graw, r.param_of + P, r.param_of + P + pb.circ.NP + 1, pb.circ.NP, grad, st);
}

// qng_energy_grad_dev and its variant on the fixed scratch: E and grad E in
// device memory, asynchronous on the context's stream.
void energy_grad_dev_call(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev, const qng_pauli_sum *ham,
                          const double *theta, qng_precision prec, void *E_dev, void *grad_dev) {
    require_ctx(ctx);
    check_prec(prec);
    validate_circuit(circ, max_qubits(prec));
    validate_theta(circ, theta);
    validate_hamiltonian(circ, ham);
    if (!E_dev || (circ->n_params > 0 && !grad_dev)) fail(QNG_E_INVALID_ARG, "output is NULL");
    reset_stats(ctx);
    Problem pb = make_problem(circ, theta, ham, ctx->opt_fusion != 0);
    dispatch(prec, [&](auto tag) {
        using R = decltype(tag);
        CallSpec spec;
        spec.grad = true;
        spec.in_dev = in_state_dev;
        CallResult r = run<R>(ctx, pb, spec);
        HIPCHECK(hipMemcpyAsync(E_dev, r.eraw, 8, hipMemcpyDeviceToDevice, ctx->stream));
        device_grad(r, pb, (double *)grad_dev, ctx->stream);
    });
}

// ------------------------------------------------------------ batched metric

// Tile width a member's plan ends up with (build_sweep_plan's clamping).
int member_tile(const Circuit &c, int opt_tile, int amp, bool f64) {
    int m = opt_tile > 0 ? opt_tile : default_tile_qubits(c.n, amp, f64);
    if (m > (f64 ? 11 : 12)) m = f64 ? 11 : 12;
    return m > c.n ? c.n : m;
}

struct BatchLayout {
    std::vector<size_t> psi, traw, graw, gout, tout, param_of, lraw_class;
    size_t lam = 0, staging = 0, partials = 0, eraw = 0, gscratch = 0, gscratch_bytes = 0;
    size_t scratch = 0, images = 0, arena = 0, spart = 0, fwd = 0, adj = 0, adj32 = 0;
    size_t total = 0;
};

struct BatchRun {
    std::vector<std::vector<int>> classes;                 // member indices per class
    std::vector<std::shared_ptr<BatchClass>> cls;
    BatchLayout L;
    char *base = nullptr;
    int64_t launches = 0;
    std::vector<double *> G, T;                            // per member: G, T in parameter order (device)
};

template <typename R>
// real_products: the sweeps keep the real parts of the metric's inner products
// (the caller needs Re G only).
BatchRun batch_metric(qng_ctx *ctx, const std::vector<Problem> &pbs, const double *const *in_states,
                      const BatchTuning &tun, bool allow_graph, bool profile, bool real_products = false) {
    const int B = (int)pbs.size();
    const int amp = 2 * (int)sizeof(R);
    const bool f64 = amp == 16 || ctx->opt_f64_regs;
    hipStream_t st = ctx->stream;
    BatchRun run;
    run.G.assign(B, nullptr);
    run.T.assign(B, nullptr);

    // register classes: members whose plans share the tile width and the
    // columns per lambda sweep (as in the single step: four for FP32 registers
    // in tiles of 11 qubits, else two for full tiles, else one; chosen
    // automatically, four only for registers of >= kBatchFourMinQubits qubits:
    // the smaller ones run launch-bound, where two columns in tiles of 12
    // measured 10 % faster)
    std::map<std::pair<int, int>, std::vector<int>> by_m;
    for (int b = 0; b < B; ++b) {
        const int maxw = ctx->opt_block == 0 && pbs[b].circ.n < kBatchFourMinQubits ? 2 : kMaxBlockWidth;
        const int w = block_width(ctx->opt_block, pbs[b].circ, tun.tile_qubits, amp, f64, maxw);
        by_m[{member_tile(pbs[b].circ, plan_tile(w, tun.tile_qubits), amp, f64), w}].push_back(b);
    }
    size_t free_b = 0, total_b = 0;
    HIPCHECK(hipMemGetInfo(&free_b, &total_b));
    const uint64_t arena_cap = (uint64_t)(free_b + ctx->ws_bytes) / 4;
    for (auto &kv : by_m) {
        const int width = kv.first.second;
        const int tile = plan_tile(width, tun.tile_qubits);
        std::vector<int32_t> key = {kv.first.first, amp, sweep_reg_mode(ctx, amp), tun.tile_qubits, tun.target_tiles,
                                    real_products ? 1 : 0, width};
        for (int b : kv.second) append_structure_key(pbs[b].circ, key);
        auto it = ctx->batch_classes.find(key);
        std::shared_ptr<BatchClass> bc;
        if (it != ctx->batch_classes.end()) {
            bc = it->second;
        } else {
            std::vector<const Circuit *> mem;
            std::vector<std::shared_ptr<const SweepPlan>> plans;
            for (int b : kv.second) {
                mem.push_back(&pbs[b].circ);
                plans.push_back(ctx->sweep_cache.get_shared(pbs[b].circ, tile, amp, 1, f64, width));
            }
            bc = std::make_shared<BatchClass>();
            bc->sched = std::make_shared<BatchSchedule>(build_batch_schedule(mem, plans, amp, tun, arena_cap));
            if (ctx->batch_classes.size() >= 64) ctx->batch_classes.clear();
            ctx->batch_classes[key] = bc;
        }
        run.classes.push_back(kv.second);
        run.cls.push_back(bc);
    }

    // workspace
    BatchLayout &L = run.L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes + 16); return o; };
    size_t vmax = 0, stage = 0;
    int nmax = 1;
    for (int b = 0; b < B; ++b) {
        const Circuit &c = pbs[b].circ;
        const size_t V = (size_t(1) << c.n) * amp;
        vmax = std::max(vmax, V);
        nmax = std::max(nmax, c.n);
        if (in_states && in_states[b]) stage = std::max(stage, (size_t(1) << c.n) * 16);
        L.psi.push_back(take(V));
        L.traw.push_back(take((size_t)c.P * 16));
        L.graw.push_back(take((size_t)c.P * 16));
        L.gout.push_back(take((size_t)c.P * c.P * 16));
        L.tout.push_back(take((size_t)c.P * 16));
        L.param_of.push_back(take(param_map_ints(c) * 4));
    }
    L.lam = take(vmax);
    size_t gsc = 0;
    if (ctx->opt_fusion)
        for (int b = 0; b < B; ++b)
            if (pbs[b].circ.P > 0)
                gsc = std::max(gsc, fused_gradient_scratch_bytes(
                                        *ctx->sweep_cache.get_gradient(pbs[b].circ, tun.tile_qubits, amp, f64), pbs[b].circ.M));
    L.gscratch = take(gsc);
    L.gscratch_bytes = gsc;
    L.staging = stage ? take(stage) : 0;
    L.partials = take((size_t)reduce_blocks(nmax) * 16);
    L.eraw = take((size_t)B * 16);
    size_t img = 0, arena = 0, spart = 0, mats = 0;
    for (size_t k = 0; k < run.cls.size(); ++k) {
        const BatchSchedule &S = *run.cls[k]->sched;
        L.lraw_class.push_back(take((size_t)S.lraw_elems * 16));
        img = std::max(img, batch_image_bytes(S));
        arena = std::max(arena, (size_t)S.arena_bytes);
        spart = std::max(spart, (size_t)S.partial_elems * 16);
        mats = std::max(mats, (size_t)S.mat_rows * 64);
    }
    L.images = take(img);
    L.arena = take(arena);
    L.spart = take(spart);
    L.fwd = take(mats);
    L.adj = take(mats);
    L.adj32 = take(mats / 2);
    L.total = off;
    char *base = ensure_workspace(ctx, L.total);
    run.base = base;

    // inputs: forward registers, parameter maps
    for (int b = 0; b < B; ++b) {
        const Circuit &c = pbs[b].circ;
        const void *src = nullptr;
        if (in_states && in_states[b]) {
            HIPCHECK(hipMemcpyAsync(base + L.staging, in_states[b], (size_t(1) << c.n) * 16, hipMemcpyHostToDevice,
                                    st));
            src = base + L.staging;
        }
        launch_init_state<R>(base + L.psi[b], c.n, src, st);
        if (c.P)
            HIPCHECK(hipMemcpyAsync(base + L.param_of[b], pbs[b].param_map.data(), pbs[b].param_map.size() * 4,
                                    hipMemcpyHostToDevice, st));
        ++ctx->stats.other_launches;
    }

    // metric phase, one register class at a time
    for (size_t k = 0; k < run.cls.size(); ++k) {
        BatchClass &bc = *run.cls[k];
        const BatchSchedule &S = *bc.sched;
        const std::vector<int> &mem = run.classes[k];
        std::vector<const Circuit *> circs;
        BatchDevice d;
        d.images = base + L.images;
        d.arena = base + L.arena;
        d.fwd_mats = (double *)(base + L.fwd);
        d.adj_mats = (double *)(base + L.adj);
        d.adj_mats32 = (float *)(base + L.adj32);
        d.partials = (double *)(base + L.spart);
        d.lraw = (double *)(base + L.lraw_class[k]);
        d.reduce_partials = (double *)(base + L.partials);
        std::vector<double> fm((size_t)S.mat_rows * 8 + 8, 0.0), am((size_t)S.mat_rows * 8 + 8, 0.0);
        for (size_t i = 0; i < mem.size(); ++i) {
            const Problem &pb = pbs[mem[i]];
            circs.push_back(&pb.circ);
            d.psi.push_back(base + L.psi[mem[i]]);
            // T right after the member's raw L: the blocks' in-pass seeds reduce into it
            d.traw.push_back(d.lraw + 2 * (S.lraw_base[i] + (int64_t)pb.circ.P * pb.circ.P));
            for (const Rot &r : pb.circ.rots) {
                const Mat2 &m = pb.fwd[r.pos];
                double *o = &fm[(size_t)(S.gate_base[i] + r.pos) * 8];
                o[0] = m.a.real(); o[1] = m.a.imag(); o[2] = m.b.real(); o[3] = m.b.imag();
                o[4] = m.c.real(); o[5] = m.c.imag(); o[6] = m.d.real(); o[7] = m.d.imag();
                const Shear sh = adjoint_shear(r.axis, pb.adj[r.pos]);
                am[(size_t)(S.gate_base[i] + r.pos) * 8 + 0] = sh.u;
                am[(size_t)(S.gate_base[i] + r.pos) * 8 + 1] = sh.w;
                if (r.ctrl >= 0) {
                    // controlled rotations: the adjoint as a plane rotation
                    const PlaneRot pl = adjoint_plane(r.axis, pb.adj[r.pos]);
                    am[(size_t)(S.gate_base[i] + r.pos) * 8 + 2] = pl.c;
                    am[(size_t)(S.gate_base[i] + r.pos) * 8 + 3] = pl.s;
                }
            }
            // the fixed rotations of rewritten Pauli strings: the forward
            // matrix and the adjoint's shear, as for the parameterised ones
            for (int pos = 0; pos < pb.circ.M; ++pos) {
                if (!pb.circ.is_fixed_rotation(pos)) continue;
                const int kind = pb.circ.gates[pos].kind;
                const Mat2 &m = pb.fwd[pos];
                double *o = &fm[(size_t)(S.gate_base[i] + pos) * 8];
                o[0] = m.a.real(); o[1] = m.a.imag(); o[2] = m.b.real(); o[3] = m.b.imag();
                o[4] = m.c.real(); o[5] = m.c.imag(); o[6] = m.d.real(); o[7] = m.d.imag();
                const Shear sh = adjoint_shear(kind == QNG_RX ? AX_X : kind == QNG_RY ? AX_Y : AX_Z, pb.adj[pos]);
                am[(size_t)(S.gate_base[i] + pos) * 8 + 0] = sh.u;
                am[(size_t)(S.gate_base[i] + pos) * 8 + 1] = sh.w;
            }
        }
        std::vector<float> am32(am.begin(), am.end());
        if (S.mat_rows) {
            HIPCHECK(hipMemcpyAsync(d.fwd_mats, fm.data(), (size_t)S.mat_rows * 64, hipMemcpyHostToDevice, st));
            HIPCHECK(hipMemcpyAsync(d.adj_mats, am.data(), (size_t)S.mat_rows * 64, hipMemcpyHostToDevice, st));
            HIPCHECK(hipMemcpyAsync(d.adj_mats32, am32.data(), (size_t)S.mat_rows * 32, hipMemcpyHostToDevice, st));
        }
        upload_batch_images(S, d, st);   // synchronises: fm, am and the images are on the device
        // stats from the schedule
        for (const BatchLaunch &bl : S.launches) {
            ++ctx->stats.sweep_launches;
            ctx->stats.sweep_tiles += bl.total_tiles;
            for (uint32_t j = 0; j < bl.n_items; ++j) {
                const LaunchItem &it = S.items[bl.item_begin + j];
                const uint64_t amps = (uint64_t)it.ntiles << S.m;
                ctx->stats.sweep_bytes += 4.0 * (double)amps * amp;
            }
            for (uint32_t j = 0; j < bl.n_tasks; ++j)
                ctx->stats.sweep_flops += sweep_flops_per_amp(1, real_products) *
                                          (double)S.tasks[bl.task_begin + j].count * (double)(1u << S.m);
        }
        ctx->stats.elements += S.elements;
        run.launches += (int64_t)S.launches.size();
        const bool graph = allow_graph && !profile && st != nullptr;
        // every device address the captured launches hold: the workspace, the
        // class's buffers and each member's registers and T (members move when
        // a batch lists its ansaetze in another order)
        std::vector<uint64_t> ptrs = {(uint64_t)(uintptr_t)base,
                                      (uint64_t)L.total,
                                      (uint64_t)(uintptr_t)d.images,
                                      (uint64_t)(uintptr_t)d.arena,
                                      (uint64_t)(uintptr_t)d.fwd_mats,
                                      (uint64_t)(uintptr_t)d.adj_mats,
                                      (uint64_t)(uintptr_t)d.adj_mats32,
                                      (uint64_t)(uintptr_t)d.partials,
                                      (uint64_t)(uintptr_t)d.lraw,
                                      (uint64_t)(uintptr_t)d.reduce_partials};
        for (size_t i = 0; i < mem.size(); ++i) {
            ptrs.push_back((uint64_t)(uintptr_t)d.psi[i]);
            ptrs.push_back((uint64_t)(uintptr_t)d.traw[i]);
        }
        if (graph) {
            if (!bc.graph || bc.graph_ptrs != ptrs) {
                if (bc.graph) {
                    HIPCHECK(hipGraphExecDestroy(bc.graph));
                    bc.graph = nullptr;
                }
                hipGraph_t g = nullptr;
                HIPCHECK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
                try {
                    enqueue_batch_metric<R>(S, circs, d, sweep_reg_mode(ctx, amp), st, nullptr, real_products);
                } catch (...) {
                    hipGraph_t junk = nullptr;
                    (void)hipStreamEndCapture(st, &junk);
                    if (junk) (void)hipGraphDestroy(junk);
                    throw;
                }
                HIPCHECK(hipStreamEndCapture(st, &g));
                hipGraphExec_t ge = nullptr;
                const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) fail(QNG_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
                bc.graph = ge;
                bc.graph_ptrs = ptrs;
            } else {
                ++ctx->stats.graph_replays;
            }
            HIPCHECK(hipGraphLaunch(bc.graph, st));
        } else {
            std::vector<hipEvent_t> ev;
            if (profile) {
                ev.resize(2 * S.launches.size());
                for (auto &e : ev) HIPCHECK(hipEventCreate(&e));
            }
            enqueue_batch_metric<R>(S, circs, d, sweep_reg_mode(ctx, amp), st, profile ? &ev : nullptr, real_products);
            if (profile) {
                HIPCHECK(hipStreamSynchronize(st));
                for (size_t li = 0; li < S.launches.size(); ++li) {
                    float ms = 0.f;
                    HIPCHECK(hipEventElapsedTime(&ms, ev[2 * li], ev[2 * li + 1]));
                    ctx->stats.sweep_ms += ms;
                }
                for (auto &e : ev) (void)hipEventDestroy(e);
            }
        }
        for (size_t i = 0; i < mem.size(); ++i) {
            const Problem &pb = pbs[mem[i]];
            double *lraw_i = d.lraw + 2 * S.lraw_base[i];   // P*P complex, dead after the unpack
            unpack_to_params(pb, lraw_i, d.traw[i], (const int *)(base + L.param_of[mem[i]]),
                             (double *)(base + L.gout[mem[i]]), (double *)(base + L.tout[mem[i]]), lraw_i,
                             run.G[mem[i]], run.T[mem[i]], st);
            ++ctx->stats.other_launches;
        }
    }
    return run;
}

// Autotuner of the batched metric: coordinate search over the tile width
// (fusion width) and the work-groups per launch, timing the whole metric phase
// of this batch; the winner is cached per batch structure.
template <typename R>
BatchTuning batch_tuning(qng_ctx *ctx, const std::vector<Problem> &pbs, const double *const *in_states) {
    const int amp = 2 * (int)sizeof(R);
    const bool f64 = amp == 16 || ctx->opt_f64_regs;
    BatchTuning fixed;
    fixed.tile_qubits = ctx->opt_tile;
    fixed.target_tiles = ctx->opt_batch_tiles > 0 ? ctx->opt_batch_tiles : 4096;
    if (!ctx->opt_autotune) return fixed;
    std::vector<int32_t> key = {amp, sweep_reg_mode(ctx, amp), ctx->opt_tile, ctx->opt_batch_tiles};
    for (const Problem &pb : pbs) append_structure_key(pb.circ, key);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return it->second;
    auto t0 = Clock::now();
    hipStream_t st = ctx->stream;
    auto time_of = [&](const BatchTuning &t) {
        hipEvent_t e0, e1;
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        const qng_stats saved = ctx->stats;
        // a first run uploads and warms; the second is timed
        batch_metric<R>(ctx, pbs, in_states, t, false, false);
        HIPCHECK(hipEventRecord(e0, st));
        batch_metric<R>(ctx, pbs, in_states, t, false, false);
        HIPCHECK(hipEventRecord(e1, st));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->stats = saved;
        return (double)ms;
    };
    std::vector<int> tiles;
    if (ctx->opt_tile > 0) tiles = {ctx->opt_tile};
    else if (f64) tiles = {10, 11};
    else tiles = {10, 11, 12};
    std::vector<int> targets;
    if (ctx->opt_batch_tiles > 0) targets = {ctx->opt_batch_tiles};
    else targets = {4096, 2048, 8192};
    BatchTuning best = fixed;
    double best_ms = 1e300;
    for (int m : tiles) {
        BatchTuning t;
        t.tile_qubits = m;
        t.target_tiles = targets[0];
        const double ms = time_of(t);
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    for (size_t k = 1; k < targets.size(); ++k) {
        BatchTuning t = best;
        t.target_tiles = targets[k];
        const double ms = time_of(t);
        if (ms < best_ms) { best_ms = ms; best = t; }
    }
    if (ctx->tuned.size() >= 64) ctx->tuned.clear();
    ctx->tuned[key] = best;
    ctx->stats.tune_ms += ms_since(t0);
    return best;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

qng_status qng_create(qng_ctx **out, int device, void *hip_stream) {
    return guarded(nullptr, [&] {
        if (!out) fail(QNG_E_INVALID_ARG, "out is NULL");
        *out = nullptr;
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
            (void)hipGetLastError();
            fail(QNG_E_DEVICE, "no HIP device available");
        }
        if (device < 0 || device >= count) fail(QNG_E_DEVICE, "device index out of range");
        HIPCHECK(hipSetDevice(device));
        // device address of the fixed scratch of qng_energy_grad_dev_noalloc
        // on this device (looked up once per device)
        HIPCHECK(noalloc_scratch_init(device));
        std::unique_ptr<qng_ctx> c(new qng_ctx);
        c->device = device;
        if (hip_stream) c->stream = (hipStream_t)hip_stream;
        else {
            HIPCHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        *out = c.release();
    });
}

void qng_destroy(qng_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *qng_last_error(const qng_ctx *ctx) {
    if (ctx) return ctx->last_error.c_str();
    return g_last_error.c_str();
}

qng_status qng_set_stream(qng_ctx *ctx, void *hip_stream) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        if (ctx->own_stream && ctx->stream) {
            HIPCHECK(hipStreamSynchronize(ctx->stream));
            HIPCHECK(hipStreamDestroy(ctx->stream));
            ctx->stream = nullptr;
            ctx->own_stream = false;
        }
        ctx->stream = (hipStream_t)hip_stream;
    });
}

qng_status qng_set_mem_limit(qng_ctx *ctx, size_t bytes) {
    return guarded(ctx, [&] {
        if (!ctx) fail(QNG_E_INVALID_ARG, "context is NULL");
        ctx->mem_limit = bytes;
    });
}

qng_status qng_set_option(qng_ctx *ctx, int option, int value) {
    return guarded(ctx, [&] {
        if (!ctx) fail(QNG_E_INVALID_ARG, "context is NULL");
        switch (option) {
        case QNG_OPT_FUSION: ctx->opt_fusion = value ? 1 : 0; break;
        case QNG_OPT_TILE_QUBITS:
            if (value < 0 || value > 14) fail(QNG_E_INVALID_ARG, "tile qubits outside [0, 14]");
            ctx->opt_tile = value;
            break;
        case QNG_OPT_COLUMN_STREAMS:
            if (value < 0) fail(QNG_E_INVALID_ARG, "column streams < 0");
            ctx->opt_streams = value;
            break;
        case QNG_OPT_PROFILE: ctx->opt_profile = value ? 1 : 0; break;
        case QNG_OPT_SMALL_N_KERNEL: ctx->opt_small = value ? 1 : 0; break;
        case QNG_OPT_F64_REGISTERS: ctx->opt_f64_regs = value ? 1 : 0; break;
        case QNG_OPT_EXACT_PRODUCTS: ctx->opt_exact_products = value ? 1 : 0; break;
        case QNG_OPT_GRAPH: ctx->opt_graph = value ? 1 : 0; break;
        case QNG_OPT_AUTOTUNE: ctx->opt_autotune = value ? 1 : 0; break;
        case QNG_OPT_BATCH_TILES:
            if (value < 0) fail(QNG_E_INVALID_ARG, "batch tiles < 0");
            ctx->opt_batch_tiles = value;
            break;
        case QNG_OPT_BLOCK_COLUMNS:
            if (value < 0 || value > kMaxBlockWidth || value == 3)
                fail(QNG_E_INVALID_ARG, "block columns must be 0 (automatic), 1, 2 or 4");
            ctx->opt_block = value;
            break;
        case QNG_OPT_METHOD:
            if (value < 0 || value > 1) fail(QNG_E_INVALID_ARG, "method must be 0 (recurrence) or 1 (derivative states)");
            ctx->opt_method = value;
            break;
        case QNG_OPT_STATE_CHUNK:
            if (value < 0) fail(QNG_E_INVALID_ARG, "state chunk < 0");
            ctx->opt_state_chunk = value;
            break;
        case QNG_OPT_METRIC_KIND:
            if (value < 0 || value > 1) fail(QNG_E_INVALID_ARG, "metric kind must be 0 (G) or 1 (L)");
            ctx->opt_metric_kind = value;
            break;
        default: fail(QNG_E_INVALID_ARG, "unknown option " + std::to_string(option));
        }
    });
}

qng_status qng_set_metric_blocks(qng_ctx *ctx, int32_t n_params, const int32_t *block_of_param) {
    return guarded(ctx, [&] {
        if (!ctx) fail(QNG_E_INVALID_ARG, "context is NULL");
        if (n_params < 0) fail(QNG_E_INVALID_ARG, "n_params < 0");
        if (n_params > 0 && !block_of_param) fail(QNG_E_INVALID_ARG, "block_of_param is NULL");
        ctx->metric_blocks.assign(block_of_param, block_of_param + (n_params > 0 ? n_params : 0));
    });
}

qng_status qng_get_stats(const qng_ctx *ctx, qng_stats *out) {
    if (!ctx || !out) return QNG_E_INVALID_ARG;
    *out = ctx->stats;
    return QNG_OK;
}

qng_status qng_synchronize(qng_ctx *ctx) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        HIPCHECK(hipStreamSynchronize(ctx->stream));
    });
}

qng_status qng_validate(const qng_circuit *circ, const double *theta, const qng_pauli_sum *ham, char *msg,
                        size_t msg_len) {
    qng_status s = guarded(nullptr, [&] {
        validate_circuit(circ, kMaxQubitsC64);
        validate_theta(circ, theta);
        if (ham) validate_hamiltonian(circ, ham);
    });
    if (msg && msg_len) {
        std::snprintf(msg, msg_len, "%s", s == QNG_OK ? "" : g_last_error.c_str());
    }
    return s;
}

qng_status qng_plan(const qng_circuit *circ, int fusion, int tile_qubits, qng_plan_info *out) {
    return guarded(nullptr, [&] {
        if (!out) fail(QNG_E_INVALID_ARG, "out is NULL");
        validate_circuit(circ, kMaxQubitsC64);
        Circuit c = compile_circuit(circ);
        *out = qng_plan_info{};
        out->elements = (int64_t)c.P * (c.P - 1) / 2;
        if (fusion && c.has_strings) {
            if (!strings_lowerable(c))
                fail(QNG_E_UNSUPPORTED, "fused sweep passes do not take Pauli-string rotations without letters");
            c = lower_strings(c);
        }
        if (!fusion) {
            for (int s = 1; s < c.P; ++s) out->ops += c.rots[s].pos - c.rots[0].pos + (s);
            out->passes = 0;
            return;
        }
        SweepPlan plan = build_sweep_plan(c, tile_qubits, 16, 1, true);
        plan.fill_info(out);
    });
}

qng_status qng_plan_export(const qng_circuit *circ, int tile_qubits, int amp_bytes, int32_t sweep, int32_t *rows,
                           int64_t cap, int64_t *n_rows) {
    return guarded(nullptr, [&] {
        if (!n_rows) fail(QNG_E_INVALID_ARG, "n_rows is NULL");
        if (amp_bytes != 8 && amp_bytes != 16) fail(QNG_E_INVALID_ARG, "amp_bytes must be 8 or 16");
        if (sweep < 0 || sweep > 4 || sweep == 3)
            fail(QNG_E_INVALID_ARG, "sweep must be 0, 2 or 4 (metric) or 1 (gradient)");
        validate_circuit(circ, kMaxQubitsC64);
        Circuit c = compile_circuit(circ);
        if (c.has_strings)
            fail(QNG_E_UNSUPPORTED, "plans of circuits with Pauli-string rotations run on a rewritten gate list "
                                    "and are not exported");
        SweepPlan plan = sweep == 1 ? build_gradient_plan(c, tile_qubits, amp_bytes, amp_bytes == 16)
                                    : build_sweep_plan(c, tile_qubits, amp_bytes, 1, amp_bytes == 16, sweep >= 2 ? sweep : 1);
        int64_t k = 0;
        auto emit = [&](const ColumnPlan &cp, size_t pi, uint64_t mask, int kind, int q0, int q1, int gate, int dest,
                        int axis) {
            if (rows && k < cap) {
                int32_t *r = rows + 10 * k;
                r[0] = cp.s;
                r[1] = (int32_t)pi;
                r[2] = kind;
                r[3] = q0;
                r[4] = q1;
                r[5] = gate;
                r[6] = dest;
                r[7] = axis;
                r[8] = (int32_t)(mask & 0x7fffffffu);
                r[9] = (int32_t)((mask >> 31) & 0x7fffffffu);
            }
            ++k;
        };
        for (const ColumnPlan &cp : plan.cols) {
            for (size_t pi = 0; pi < cp.passes.size(); ++pi) {
                const HostPass &hp = cp.passes[pi];
                uint64_t mask = 0;
                for (uint8_t q : hp.tile) mask |= uint64_t(1) << q;
                for (const DevOp &op : hp.ops) {
                    if (op.type == OP_XPOSE) continue;
                    if (op.type == OP_SEED || op.type == OP_CSEED) {
                        emit(cp, pi, mask, 3, op.q0, op.type == OP_CSEED ? op.q1 : -1, -1, hp.slot_dest[op.slot],
                             op.axis);
                        continue;
                    }
                    const bool cprod = op.type == OP_PRODCROT || op.type == OP_PRODC || op.type == OP_PRODCDIAG ||
                                       op.type == OP_PRODCZ;
                    const bool prod = cprod || op.type == OP_PRODROT || op.type == OP_PROD || op.type == OP_ZSUM ||
                                      op.type == OP_PRODZ || op.type == OP_PRODDIAG;
                    const bool adj = op.type == OP_ROT || op.type == OP_PRODROT || op.type == OP_CNOT ||
                                     op.type == OP_CZ || op.type == OP_DIAG || op.type == OP_PRODDIAG ||
                                     op.type == OP_CROT || op.type == OP_PRODCROT || op.type == OP_CDIAG ||
                                     op.type == OP_PRODCDIAG;
                    if (!prod) {
                        // controlled rotations as in the gate list: q0 the control, q1 the target
                        if (op.type == OP_CROT || op.type == OP_CDIAG)
                            emit(cp, pi, mask, 0, op.q1, op.q0, op.gate, -1, -1);
                        else
                            emit(cp, pi, mask, 0, op.q0, (op.type == OP_CNOT || op.type == OP_CZ) ? op.q1 : -1,
                                 op.gate, -1, -1);
                        continue;
                    }
                    // one row per active phi register; the adjoint (if any) rides on the last
                    const int nprod = plan.width - op.aux;
                    for (int b = 0; b < nprod; ++b) {
                        const bool last = b + 1 == nprod;
                        emit(cp, pi, mask, (last && adj) ? 1 : 2, op.q0, cprod ? op.q1 : -1,
                             (last && adj) ? op.gate : -1, hp.slot_dest[op.slot + b], op.axis);
                    }
                }
            }
        }
        *n_rows = k;
    });
}

qng_status qng_solve_shifted(int32_t P, const double *G, double eps, const double *b, double *x) {
    return guarded(nullptr, [&] {
        if (P < 0 || (P > 0 && (!G || !b || !x))) fail(QNG_E_INVALID_ARG, "bad arguments");
        validate_scalar(eps, "eps");
        if (eps < 0) fail(QNG_E_INVALID_ARG, "eps < 0");
        qng::solve_shifted(P, G, eps, b, x);
    });
}

qng_status qng_metric(qng_ctx *ctx, const qng_circuit *circ, const double *in_state, const double *theta,
                      qng_precision prec, double *G_out, double *T_out) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        validate_circuit(circ, max_qubits(prec));
        validate_theta(circ, theta);
        if (circ->n_params > 0 && !G_out) fail(QNG_E_INVALID_ARG, "G_out is NULL");
        check_in_state_host(circ->n_qubits, in_state);
        reset_stats(ctx);
        Problem pb = make_problem(circ, theta, nullptr, ctx->opt_fusion != 0);
        apply_metric_settings(ctx, pb);
        const int NP = pb.circ.NP;
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            CallSpec spec;
            spec.metric = true;
            spec.in_host = in_state;
            spec.host_call = true;
            CallResult r = run<R>(ctx, pb, spec);
            if (NP) {
                HIPCHECK(hipMemcpyAsync(G_out, r.G, (size_t)NP * NP * 16, hipMemcpyDeviceToHost, ctx->stream));
                if (T_out) HIPCHECK(hipMemcpyAsync(T_out, r.T, (size_t)NP * 16, hipMemcpyDeviceToHost, ctx->stream));
            }
            HIPCHECK(hipStreamSynchronize(ctx->stream));
        });
    });
}

qng_status qng_energy_grad(qng_ctx *ctx, const qng_circuit *circ, const double *in_state, const qng_pauli_sum *ham,
                           const double *theta, qng_precision prec, double *E_out, double *grad_out) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        validate_circuit(circ, max_qubits(prec));
        validate_theta(circ, theta);
        validate_hamiltonian(circ, ham);
        if (!E_out || (circ->n_params > 0 && !grad_out)) fail(QNG_E_INVALID_ARG, "output is NULL");
        check_in_state_host(circ->n_qubits, in_state);
        reset_stats(ctx);
        Problem pb = make_problem(circ, theta, ham, ctx->opt_fusion != 0);
        const int P = pb.circ.P;
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            CallSpec spec;
            spec.grad = true;
            spec.in_host = in_state;
            spec.host_call = true;
            CallResult r = run<R>(ctx, pb, spec);
            std::vector<double> graw(2 * (size_t)P + 2), e(2);
            HIPCHECK(hipMemcpyAsync(graw.data(), r.graw, (size_t)P * 16, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHECK(hipMemcpyAsync(e.data(), r.eraw, 16, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHECK(hipStreamSynchronize(ctx->stream));
            *E_out = e[0];
            host_unpack_grad(graw, pb, grad_out);
        });
    });
}

qng_status qng_step(qng_ctx *ctx, const qng_circuit *circ, const double *in_state, const qng_pauli_sum *ham,
                    const double *theta, double dt, double tikhonov, qng_precision prec, double *dtheta_out,
                    double *G_out, double *grad_out, double *E_out) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        validate_circuit(circ, max_qubits(prec));
        validate_theta(circ, theta);
        validate_hamiltonian(circ, ham);
        validate_scalar(dt, "dt");
        validate_scalar(tikhonov, "tikhonov");
        if (tikhonov < 0) fail(QNG_E_INVALID_ARG, "tikhonov < 0");
        if (circ->n_params > 0 && !dtheta_out) fail(QNG_E_INVALID_ARG, "dtheta_out is NULL");
        check_in_state_host(circ->n_qubits, in_state);
        reset_stats(ctx);
        Problem pb = make_problem(circ, theta, ham, ctx->opt_fusion != 0);
        apply_metric_settings(ctx, pb);
        const int P = pb.circ.P, NP = pb.circ.NP;
        std::vector<double> G(2 * (size_t)NP * NP + 2), graw(2 * (size_t)P + 2), e(2), grad(NP + 1);
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            CallSpec spec;
            spec.metric = true;
            spec.grad = true;
            spec.in_host = in_state;
            spec.host_call = true;
            // the solve reads Re G only: without a G output, the metric's
            // inner products keep their real parts
            spec.real_products = G_out == nullptr;
            CallResult r = run<R>(ctx, pb, spec);
            if (P) {
                HIPCHECK(hipMemcpyAsync(G.data(), r.G, (size_t)NP * NP * 16, hipMemcpyDeviceToHost, ctx->stream));
                HIPCHECK(hipMemcpyAsync(graw.data(), r.graw, (size_t)P * 16, hipMemcpyDeviceToHost, ctx->stream));
            }
            HIPCHECK(hipMemcpyAsync(e.data(), r.eraw, 16, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHECK(hipStreamSynchronize(ctx->stream));
        });
        host_unpack_grad(graw, pb, grad.data());
        auto t0 = Clock::now();
        std::vector<double> b(NP + 1);
        for (int i = 0; i < NP; ++i) b[i] = -dt * grad[i];
        std::vector<double> x(NP + 1);
        if (NP) qng::solve_shifted(NP, G.data(), tikhonov, b.data(), x.data());
        ctx->stats.solve_ms = ms_since(t0);
        if (NP) std::memcpy(dtheta_out, x.data(), (size_t)NP * 8);
        if (G_out && NP) std::memcpy(G_out, G.data(), (size_t)NP * NP * 16);
        if (grad_out && NP) std::memcpy(grad_out, grad.data(), (size_t)NP * 8);
        if (E_out) *E_out = e[0];
    });
}

qng_status qng_step_batched(qng_ctx *ctx, int32_t B, const qng_circuit *circs, const double *const *in_states,
                            const qng_pauli_sum *hams, const double *const *thetas, double dt, double tikhonov,
                            qng_precision prec, double *const *dtheta_out, double *const *G_out,
                            double *const *grad_out, double *E_out) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        if (B < 0 || (B > 0 && (!circs || !hams || !thetas || !dtheta_out)))
            fail(QNG_E_INVALID_ARG, "bad batch arguments");
        validate_scalar(dt, "dt");
        validate_scalar(tikhonov, "tikhonov");
        if (tikhonov < 0) fail(QNG_E_INVALID_ARG, "tikhonov < 0");
        for (int b = 0; b < B; ++b) {
            try {
                validate_circuit(&circs[b], max_qubits(prec));
                validate_theta(&circs[b], thetas[b]);
                validate_hamiltonian(&circs[b], &hams[b]);
                if (circs[b].n_params > 0 && !dtheta_out[b]) fail(QNG_E_INVALID_ARG, "dtheta_out is NULL");
                check_in_state_host(circs[b].n_qubits, in_states ? in_states[b] : nullptr);
            } catch (const Error &e) {
                fail(e.status, "ansatz " + std::to_string(b) + ": " + e.msg);
            }
        }
        reset_stats(ctx);
        if (B == 0) return;
        std::vector<Problem> pbs;
        pbs.reserve(B);
        if (!ctx->metric_blocks.empty())
            fail(QNG_E_INVALID_ARG, "the block-diagonal metric is not available in qng_step_batched");
        for (int b = 0; b < B; ++b) {
            // Pauli-string rotations rewritten onto gates the passes take
            pbs.push_back(make_problem(&circs[b], thetas[b], &hams[b], true));
            if (pbs.back().circ.has_strings)
                fail(QNG_E_UNSUPPORTED, "ansatz " + std::to_string(b) +
                                            ": a Pauli-string rotation with no letter is not available in "
                                            "qng_step_batched");
            apply_metric_settings(ctx, pbs.back());
        }
        std::vector<std::vector<double>> G(B), graw(B);
        std::vector<double> E(2 * (size_t)B);
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            const BatchTuning tun = batch_tuning<R>(ctx, pbs, in_states);
            ctx->stats.tile_qubits = tun.tile_qubits;
            ctx->stats.target_tiles = tun.target_tiles;
            auto t0 = Clock::now();
            // the solves read Re G only: without G outputs the sweeps keep real parts
            bool want_G = false;
            for (int b = 0; G_out && b < B; ++b) want_G = want_G || G_out[b] != nullptr;
            BatchRun run = batch_metric<R>(ctx, pbs, in_states, tun, ctx->opt_graph != 0, ctx->opt_profile != 0,
                                           !want_G);
            HIPCHECK(hipStreamSynchronize(ctx->stream));
            ctx->stats.metric_ms = ms_since(t0);
            t0 = Clock::now();
            const BatchLayout &L = run.L;
            char *base = run.base;
            const size_t amp = 2 * sizeof(R);
            for (int b = 0; b < B; ++b) {
                const Problem &pb = pbs[b];
                Engine<R> e(ctx, pb, ctx->stream, base + L.psi[b], base + L.lam, nullptr,
                            (size_t(1) << pb.circ.n) * amp, (double *)(base + L.partials), nullptr,
                            (double *)(base + L.traw[b]), (double *)(base + L.graw[b]),
                            (double *)(base + L.eraw) + 2 * b);
                std::shared_ptr<const SweepPlan> gp;
                if (ctx->opt_fusion && pb.circ.P > 0) {
                    gp = ctx->sweep_cache.get_gradient(pb.circ, tun.tile_qubits, (int)amp, amp == 16 || ctx->opt_f64_regs);
                    e.gplan = gp.get();
                    e.gscratch = base + L.gscratch;
                    e.gscratch_bytes = L.gscratch_bytes;
                    e.reg_mode = sweep_reg_mode(ctx, amp);
                }
                e.finish_energy_grad(batch_final_pos(pb.circ), true, nullptr);
            }
            for (int b = 0; b < B; ++b) {
                const int P = pbs[b].circ.P, NP = pbs[b].circ.NP;
                G[b].assign(2 * (size_t)NP * NP + 2, 0.0);
                graw[b].assign(2 * (size_t)P + 2, 0.0);
                if (P) {
                    HIPCHECK(hipMemcpyAsync(G[b].data(), run.G[b], (size_t)NP * NP * 16, hipMemcpyDeviceToHost,
                                            ctx->stream));
                    HIPCHECK(hipMemcpyAsync(graw[b].data(), base + L.graw[b], (size_t)P * 16, hipMemcpyDeviceToHost,
                                            ctx->stream));
                }
            }
            HIPCHECK(hipMemcpyAsync(E.data(), base + L.eraw, (size_t)B * 16, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHECK(hipStreamSynchronize(ctx->stream));
            ctx->stats.grad_ms = ms_since(t0);
        });
        auto t0 = Clock::now();
        // every member is solved before any output is written, so a member
        // whose shifted metric is not positive definite leaves all outputs
        // untouched
        std::vector<std::vector<double>> grads(B), xs(B);
        for (int b = 0; b < B; ++b) {
            const int NP = pbs[b].circ.NP;
            std::vector<double> rhs(NP + 1);
            grads[b].assign(NP + 1, 0.0);
            xs[b].assign(NP + 1, 0.0);
            host_unpack_grad(graw[b], pbs[b], grads[b].data());
            for (int i = 0; i < NP; ++i) rhs[i] = -dt * grads[b][i];
            if (NP) {
                try {
                    qng::solve_shifted(NP, G[b].data(), tikhonov, rhs.data(), xs[b].data());
                } catch (const Error &e) {
                    fail(e.status, "ansatz " + std::to_string(b) + ": " + e.msg);
                }
            }
        }
        for (int b = 0; b < B; ++b) {
            const int NP = pbs[b].circ.NP;
            if (NP) {
                std::memcpy(dtheta_out[b], xs[b].data(), (size_t)NP * 8);
                if (G_out && G_out[b]) std::memcpy(G_out[b], G[b].data(), (size_t)NP * NP * 16);
                if (grad_out && grad_out[b]) std::memcpy(grad_out[b], grads[b].data(), (size_t)NP * 8);
            }
            if (E_out) E_out[b] = E[2 * b];
        }
        ctx->stats.solve_ms = ms_since(t0);
    });
}

qng_status qng_metric_dev(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev, const double *theta,
                          qng_precision prec, void *G_dev, void *T_dev) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        validate_circuit(circ, max_qubits(prec));
        validate_theta(circ, theta);
        if (circ->n_params > 0 && !G_dev) fail(QNG_E_INVALID_ARG, "G_dev is NULL");
        reset_stats(ctx);
        Problem pb = make_problem(circ, theta, nullptr, ctx->opt_fusion != 0);
        apply_metric_settings(ctx, pb);
        const int NP = pb.circ.NP;
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            CallSpec spec;
            spec.metric = true;
            spec.in_dev = in_state_dev;
            CallResult r = run<R>(ctx, pb, spec);
            if (NP) {
                HIPCHECK(hipMemcpyAsync(G_dev, r.G, (size_t)NP * NP * 16, hipMemcpyDeviceToDevice, ctx->stream));
                if (T_dev) HIPCHECK(hipMemcpyAsync(T_dev, r.T, (size_t)NP * 16, hipMemcpyDeviceToDevice, ctx->stream));
            }
        });
    });
}

qng_status qng_energy_dev(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev, const qng_pauli_sum *ham,
                          const double *theta, qng_precision prec, void *E_dev, void *psi_dev) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        validate_circuit(circ, max_qubits(prec));
        validate_theta(circ, theta);
        validate_hamiltonian(circ, ham);
        if (!E_dev || !psi_dev) fail(QNG_E_INVALID_ARG, "output is NULL");
        reset_stats(ctx);
        Problem pb = make_problem(circ, theta, ham);
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            CallSpec spec;
            spec.in_dev = in_state_dev;
            spec.psi_out_dev = psi_dev;
            CallResult r = run<R>(ctx, pb, spec);
            HIPCHECK(hipMemcpyAsync(E_dev, r.eraw, 8, hipMemcpyDeviceToDevice, ctx->stream));
        });
    });
}

qng_status qng_energy_grad_from_state_dev(qng_ctx *ctx, const qng_circuit *circ, const qng_pauli_sum *ham,
                                          const double *theta, qng_precision prec, const void *psi_dev,
                                          void *grad_dev) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        validate_circuit(circ, max_qubits(prec));
        validate_theta(circ, theta);
        validate_hamiltonian(circ, ham);
        if (!psi_dev || (circ->n_params > 0 && !grad_dev)) fail(QNG_E_INVALID_ARG, "pointer is NULL");
        reset_stats(ctx);
        Problem pb = make_problem(circ, theta, ham, ctx->opt_fusion != 0);
        const int P = pb.circ.P;
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            CallSpec spec;
            spec.grad = true;
            spec.psi_final_dev = psi_dev;
            CallResult r = run<R>(ctx, pb, spec);
            (void)P;
            device_grad(r, pb, (double *)grad_dev, ctx->stream);
        });
    });
}

qng_status qng_energy_grad_dev(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev,
                               const qng_pauli_sum *ham, const double *theta, qng_precision prec, void *E_dev,
                               void *grad_dev) {
    return guarded(ctx, [&] { energy_grad_dev_call(ctx, circ, in_state_dev, ham, theta, prec, E_dev, grad_dev); });
}

qng_status qng_energy_grad_dev_noalloc(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev,
                                       const qng_pauli_sum *ham, const double *theta, qng_precision prec,
                                       void *E_dev, void *grad_dev) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        char *fixed = (char *)noalloc_scratch(ctx->device);
        if (!fixed) fail(QNG_E_DEVICE, "the fixed scratch of this device was not looked up (qng_create)");
        // the context's own workspace is left alone; every buffer of this call
        // is carved from the fixed scratch
        struct Use {
            qng_ctx *c;
            ~Use() {
                c->fixed_ws = nullptr;
                c->fixed_ws_bytes = 0;
            }
        } use{ctx};
        ctx->fixed_ws = fixed;
        ctx->fixed_ws_bytes = kNoallocScratchBytes;
        energy_grad_dev_call(ctx, circ, in_state_dev, ham, theta, prec, E_dev, grad_dev);
    });
}

qng_status qng_step_dev(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev, const qng_pauli_sum *ham,
                        const double *theta, double dt, double tikhonov, qng_precision prec, void *dtheta_dev,
                        void *G_dev, void *grad_dev, void *E_dev, int32_t *status_dev) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        validate_circuit(circ, max_qubits(prec));
        validate_theta(circ, theta);
        validate_hamiltonian(circ, ham);
        validate_scalar(dt, "dt");
        validate_scalar(tikhonov, "tikhonov");
        if (tikhonov < 0) fail(QNG_E_INVALID_ARG, "tikhonov < 0");
        if (circ->n_params > 0 && !dtheta_dev) fail(QNG_E_INVALID_ARG, "dtheta_dev is NULL");
        reset_stats(ctx);
        Problem pb = make_problem(circ, theta, ham, ctx->opt_fusion != 0);
        apply_metric_settings(ctx, pb);
        const int NP = pb.circ.NP;
        hipStream_t st = ctx->stream;
        int32_t solve_status = 0;
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            CallSpec spec;
            spec.metric = true;
            spec.grad = true;
            spec.in_dev = in_state_dev;
            spec.device_solve = true;
            // the solve reads Re G only: without a G output the metric's inner
            // products keep their real parts
            spec.real_products = G_dev == nullptr;
            CallResult r = run<R>(ctx, pb, spec);
            // solve workspace: A (NP*NP), y, x, grad (NP each), status
            double *A = (double *)r.solve;
            double *y = A + (size_t)NP * NP, *x = y + NP, *grad = x + NP;
            int32_t *status = (int32_t *)(grad + NP);
            device_grad(r, pb, grad, st);
            if (NP) launch_shifted_solve(r.G, NP, tikhonov, grad, dt, A, y, x, status, st);
            else HIPCHECK(hipMemsetAsync(status, 0, sizeof(int32_t), st));
            // every output follows the solve's status: nothing is written when
            // Re G + eps I is not positive definite
            launch_copy_if_ok(status, x, (double *)dtheta_dev, NP, st);
            if (G_dev) launch_copy_if_ok(status, r.G, (double *)G_dev, 2 * (int64_t)NP * NP, st);
            if (grad_dev) launch_copy_if_ok(status, grad, (double *)grad_dev, NP, st);
            if (E_dev) launch_copy_if_ok(status, r.eraw, (double *)E_dev, 1, st);
            if (status_dev) {
                HIPCHECK(hipMemcpyAsync(status_dev, status, sizeof(int32_t), hipMemcpyDeviceToDevice, st));
            } else {
                HIPCHECK(hipMemcpyAsync(&solve_status, status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
                HIPCHECK(hipStreamSynchronize(st));
            }
        });
        if (!status_dev && solve_status != 0)
            fail(QNG_E_NOT_SPD, "Re G + eps I is not positive definite (device solve); no output was written");
    });
}

qng_status qng_clone_state_dev(qng_ctx *ctx, int32_t n_qubits, qng_precision prec, const void *src_dev,
                               void *dst_dev) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        if (n_qubits < 0 || n_qubits > max_qubits(prec)) fail(QNG_E_INVALID_ARG, "n_qubits out of range");
        if (!src_dev || !dst_dev) fail(QNG_E_INVALID_ARG, "state pointer is NULL");
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            launch_copy<R>(src_dev, dst_dev, n_qubits, ctx->stream);
        });
    });
}

qng_status qng_apply_circuit_dev(qng_ctx *ctx, const qng_circuit *circ, const double *theta, qng_precision prec,
                                 void *state_dev) {
    return guarded(ctx, [&] {
        require_ctx(ctx);
        check_prec(prec);
        validate_circuit(circ, max_qubits(prec));
        validate_theta(circ, theta);
        if (!state_dev) fail(QNG_E_INVALID_ARG, "state_dev is NULL");
        Problem pb = make_problem(circ, theta, nullptr);
        dispatch(prec, [&](auto tag) {
            using R = decltype(tag);
            for (int pos = 0; pos < pb.circ.M; ++pos) apply_gate<R>(pb, pos, false, state_dev, nullptr, ctx->stream);
        });
    });
}

}  // extern "C"
