// sweep.hpp -- fused, tiled execution of the backward sweeps of the metric.
//
// Column s of the recurrence (Sec. 2 recurrences, Sec. 3 Alg. 1; see api.cpp)
// sweeps two registers lambda, phi backwards through the same adjoint gates
// and takes one Pauli-weighted inner product <lambda|sigma_r|phi> per earlier
// rotation r.  Executed one primitive at a time this reads and writes both
// registers for every gate (the paper's own primitive-level schedule).  Here
// the sweep of a column is cut into *passes*: a pass fixes a set of m qubits
// (its tile), and every operation of the pass acts only on those qubits, so
// the register splits into 2^(n-m) independent tiles of 2^m amplitudes.  A
// work-group loads one tile of lambda and phi into LDS, runs the pass's whole
// operation list on-chip, writes the tile back and emits per-tile partial sums
// of the inner products.  One pass reads and writes each register once.
//
// Reordering.  Operations of the sweep are reordered only when they commute.
// Every operation acts on each of its qubits through one Pauli "type": RX and
// a CNOT target are X-type, RY is Y-type, RZ, CZ and a CNOT control are
// Z-type, and the inner product <lambda|sigma|phi> is of sigma's type on its
// qubit (both registers receive the same gates, so <V lambda|sigma|V phi> =
// <lambda|sigma|phi> whenever V commutes with sigma).  Two operations commute
// when their types agree on every shared qubit.
//
// What a tile can execute: X/Y rotations and X/Y inner products on tile
// qubits; RZ on tile qubits; a CNOT whose target is in the tile (its control
// may lie outside: then it is fixed per tile); a CZ with at least one qubit in
// the tile; a Z inner product on any qubit (outside the tile its value is
// +-<lambda|phi> restricted to the tile, and that restricted sum is invariant
// under every in-tile operation, so it is taken once when the tile is loaded).
// RZ and CZ factors that are constant over a tile are never applied early:
// they stay pending until one of their qubits enters a tile, which is always
// before any operation they do not commute with.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <map>
#include <memory>
#include <vector>

#include "circuit.hpp"
#include "kernels.hpp"

namespace qng {

enum : uint8_t {
    OP_ROT = 0,       // X/Y rotation adjoint (stored matrix) on register position b0
    OP_PRODROT = 1,   // X/Y inner product on register position b0, then the rotation adjoint
    OP_PROD = 2,      // X/Y inner product <A|sigma|B> on register position b0
    OP_CNOT = 3,      // CNOT adjoint: target register position b0, control location b1 (qubit q0)
    OP_CZ = 4,        // sign (-1)^{x_a x_b}: locations b0 (qubit q0), b1 (qubit q1)
    OP_ZSUM = 5,      // Z inner product on qubit q0 outside the tile: +-<A|B>_tile
    OP_DIAG = 6,      // RZ adjoint diag(m00, m11) on location b0
    OP_PRODZ = 7,     // Z inner product on location b0
    OP_PRODDIAG = 8,  // Z inner product on location b0, then the RZ adjoint there
    OP_XPOSE = 9,     // exchange through LDS to the thread mapping `aux`
    OP_SEED = 10,     // column block: phi register `aux` <- sigma lambda (sigma on qubit q0, location b0),
                      // then <lambda|phi> into the op's slot
    // controlled rotations (generator |1><1|_c (x) sigma_t): target qubit q0 at
    // location b0, control qubit q1 at location b1
    OP_CROT = 11,     // X/Y controlled rotation adjoint, target on register position b0
    OP_PRODCROT = 12, // X/Y inner product <A|K|B>, then the adjoint
    OP_PRODC = 13,    // X/Y inner product <A|K|B>
    OP_CDIAG = 14,    // CRZ adjoint (target at any location in the tile)
    OP_PRODCDIAG = 15,   // Z inner product <A|K|B>, then the CRZ adjoint
    OP_PRODCZ = 16,   // Z inner product <A|K|B>
    OP_CSEED = 17     // column block: phi register `aux` <- K lambda, then <lambda|phi> into the slot
};

// Device op codes.  In the flattened device images (SweepPlan::dev_ops and
// the batch images) DevOp::type holds one of these codes instead of the OP_*
// kind: the register position, the Pauli axis and where a control or a Z bit
// lives are resolved on the host, so the kernel runs one straight-line path
// per code.  "+ j" is the register position (< 4).
enum : uint8_t {
    OPC_ROT_X = 0,            // + j
    OPC_ROT_Y = 4,            // + j
    OPC_PRODROT_X = 8,        // + j
    OPC_PRODROT_Y = 12,       // + j
    OPC_PROD_X = 16,          // + j
    OPC_PROD_Y = 20,          // + j
    OPC_PRODZ_REG = 24,       // + j
    OPC_PRODZ_THR = 28,       // Z bit on thread position b0 & 15
    OPC_PRODZ_BASE = 29,      // Z bit of the tile base (qubit q0)
    OPC_DIAG_REG = 32,        // + j
    OPC_DIAG_THR = 36,
    OPC_DIAG_BASE = 37,
    OPC_PRODDIAG_REG = 40,    // + j
    OPC_PRODDIAG_THR = 44,
    OPC_PRODDIAG_BASE = 45,
    OPC_CNOT_REG = 48,        // + 4 j + k: target register position j, control register position k
    OPC_CNOT_THR = 64,        // + j: control on thread position b1 & 15
    OPC_CNOT_BASE = 68,       // + j: control = bit q0 of the tile base
    OPC_CZ = 72,
    OPC_ZSUM = 73,
    OPC_XPOSE = 74,
    OPC_SEED = 75,
    // controlled rotations (second handler word, HB2_* below)
    OPC_CROT_X = 76,          // + j
    OPC_CROT_Y = 80,          // + j
    OPC_PRODCROT_X = 84,      // + j
    OPC_PRODCROT_Y = 88,      // + j
    OPC_PRODC_X = 92,         // + j
    OPC_PRODC_Y = 96,         // + j
    OPC_CDIAG = 100,
    OPC_PRODCDIAG = 101,
    OPC_PRODCZ = 102,
    OPC_CSEED = 103
};

// Location of a local bit in the current thread mapping: a register position
// (< kLocThread), a thread position (kLocThread | t), or a bit of the tile base
// (kLocBase: qubit given separately).
constexpr uint8_t kLocThread = 0x10;
constexpr uint8_t kLocBase = 0xFF;
constexpr int kMaxSlots = 256;      // inner products per pass
constexpr int kMaxTileQubits = 13;
constexpr int kMaxRest = 24;        // qubits outside a tile
constexpr int kMaxBlockWidth = 4;   // columns sharing one lambda sweep
constexpr int kDefaultBlockWidth = 2;   // measured at n = 26: 8-11 % less sweep time than 1

struct DevOp {  // 32 bytes
    uint8_t type, b0, b1, axis;
    uint16_t slot;    // inner products: slot of the first active phi register (one slot per active phi)
    uint8_t q0, q1;   // qubits (global) the operation acts on
    int32_t gate;     // gate position: row of the matrix table
    int32_t aux;      // OP_XPOSE: mapping index; inner products: first active phi register;
                      // OP_SEED: the phi register seeded
    uint32_t hlo, hhi;   // device images: one-hot handler bit (HB_* below), low and high word
    uint32_t h2;         // device images: one-hot bit of the controlled-rotation handlers (HB2_*), or 0
    uint32_t pad1;
};

struct DevPass {  // 64 bytes, read through a pointer with scalar loads
    uint32_t op_begin, n_ops;
    uint16_t n_slots;
    uint8_t m, n;
    uint8_t nrest, has_zsum, rb, pad0;
    uint32_t map_load;   // thread mapping used to load the tile
    uint32_t pad1;
    uint8_t tile_q[16];  // local bit -> qubit
    uint8_t rest_q[kMaxRest];
};

// Thread mapping of a tile: position p < rb is register bit p of every thread;
// position rb + t is bit t of the thread index; pos[p] = local bit held there.
struct DevMap {
    uint8_t pos[16];
};
static_assert(sizeof(DevPass) == 64, "DevPass layout");

// Device op code of a planned operation (OPC_* above).
uint8_t device_opcode(const DevOp &op);

// Handler bits of the kernel's op loop.  Every op carries exactly one bit
// (one-hot, read from memory), and the kernel runs each handler under its own
// test of that word: a chain of independent tests, rather than one multi-way
// branch, lets the compiler keep the register tile in place through the loop
// (at a multi-way merge it assigns the tile new registers and copies it every
// iteration).  Groups of bits are tested first.
enum : int {
    HB_ROT_X = 0,            // + j
    HB_ROT_Y = 4,            // + j
    HB_PRODROT_X = 8,        // + j
    HB_PRODROT_Y = 12,       // + j
    HB_PROD_X = 16,          // + j
    HB_PROD_Y = 20,          // + j
    HB_PRODZ_REG = 24,       // + j
    HB_PRODZ_UNI = 28,       // Z bit held by the thread index or the tile base
    HB_XPOSE = 29,
    HB_CZ = 30,
    HB_ZSUM = 31,
    HB_DIAG_REG = 32,        // + j
    HB_DIAG_UNI = 36,
    HB_PRODDIAG_REG = 37,    // + j
    HB_PRODDIAG_UNI = 41,
    HB_CNOT_REG = 42,        // + index of (j, k), k != j: 3 j + (k < j ? k : k - 1)
    HB_CNOT_THR = 54,        // + j
    HB_CNOT_BASE = 58,       // + j
    HB_SEED = 62
};
int device_handler(uint8_t opcode);
// Handler bits of the controlled-rotation ops, in the second handler word that
// only the kernels built for circuits with controlled rotations test.
enum : int {
    HB2_CROT_X = 0,          // + j
    HB2_CROT_Y = 4,          // + j
    HB2_PRODCROT_X = 8,      // + j
    HB2_PRODCROT_Y = 12,     // + j
    HB2_PRODC_X = 16,        // + j
    HB2_PRODC_Y = 20,        // + j
    HB2_CDIAG = 24,
    HB2_PRODCDIAG = 25,
    HB2_PRODCZ = 26,
    HB2_CSEED = 27
};
// -1 for an op code of the first word
int device_handler2(uint8_t opcode);
static_assert(sizeof(DevOp) == 32, "DevOp layout");
static_assert(sizeof(DevMap) == 16, "DevMap layout");

struct HostPass {
    std::vector<uint8_t> tile;          // local bit -> qubit
    std::vector<DevOp> ops;             // includes OP_XPOSE (aux = index into maps)
    std::vector<int32_t> slot_dest;     // per slot: (rotation r) * P + column s
    std::vector<DevMap> maps;           // thread mappings of this pass
    int map_load = 0;                   // index into maps
    int rb = 0;                         // register bits per thread
    int transposes = 0;
};

// A column block: the columns s - width + 1 .. s (those >= 1) share one
// lambda sweep.  Column s (phi register width - 1) is seeded before the first
// pass; each lower column s_b (phi register b) is seeded inside the sweep
// (OP_SEED) where lambda reaches y_{s_b}.  With width 1 a block is one column.
struct ColumnPlan {
    int s = 0;                          // top column of the block
    std::vector<HostPass> passes;
};

struct SweepPlan {
    int n = 0, m = 0, carriers = 0, P = 0;
    int width = 1;                      // columns per block (phi registers per sweep)
    std::vector<ColumnPlan> cols;       // blocks, top columns P-1, P-1-width, ... (>= 1)
    // flattened device images
    std::vector<DevPass> dev_passes;
    std::vector<DevOp> dev_ops;
    std::vector<DevMap> dev_maps;
    int rb = 0;                         // register bits per thread (all passes)
    bool ctrl = false;                  // some op is a controlled rotation (kernels with the second handler word)
    int64_t transposes = 0;
    std::vector<int64_t> col_pass_begin;   // per column: index of its first pass in dev_passes
    int64_t total_passes = 0, total_ops = 0, max_slots = 0, load_maps = 0;
    // Metric plans: the forward register's way between block tops as tile
    // passes (a plan of width 0 whose column k applies the gates at positions
    // from rots[0].pos, then from the previous top's rotation, up to block k's
    // top rotation, in order), or null where the passes cannot take it
    // (controlled rotations).
    std::shared_ptr<const SweepPlan> forward;

    size_t device_bytes() const;        // passes + ops (the rest is per call)
    void fill_info(qng_plan_info *out) const;
};

// Register bits per thread for a tile of m qubits (256 threads per tile).
int register_bits(int m, int amp_bytes);

// Build the plan of all columns.  tile_qubits = 0 picks the default: 12 for
// FP32 registers, 11 for FP64 registers (at most n).
// reg_f64: tiles are computed in FP64 registers (always for complex128).
// width: columns per block (1 or kMaxBlockWidth).  Destinations: element
// (r, s) -> r * P + s; T_s of a column seeded inside the sweep -> P * P + s.
// rot_block (nullable, width 1): block id per rotation -- only the elements
// inside a block are planned (block-diagonal approximation).
SweepPlan build_sweep_plan(const Circuit &c, int tile_qubits, int amp_bytes, int small, bool reg_f64,
                           int width = 1, const std::vector<int> *rot_block = nullptr);
int default_tile_qubits(int n, int amp_bytes, bool reg_f64);

// Plan of the energy gradient's reverse sweep (one column, s = P): registers
// lambda = H psi and phi = psi swept back from the last gate; the inner product
// <lambda|sigma_r|phi> of rotation r goes to destination r.
SweepPlan build_gradient_plan(const Circuit &c, int tile_qubits, int amp_bytes, bool reg_f64);

struct SweepCache {
    std::map<std::vector<int32_t>, std::shared_ptr<SweepPlan>> plans;
    const SweepPlan &get(const Circuit &c, int tile_qubits, int amp_bytes, int small, bool reg_f64, int width = 1,
                         const std::vector<int> *rot_block = nullptr) {
        return *get_shared(c, tile_qubits, amp_bytes, small, reg_f64, width, rot_block);
    }
    // The plan stays alive while the caller holds the pointer, even if the
    // cache evicts it.
    std::shared_ptr<const SweepPlan> get_shared(const Circuit &c, int tile_qubits, int amp_bytes, int small,
                                                bool reg_f64, int width = 1,
                                                const std::vector<int> *rot_block = nullptr);
    std::shared_ptr<const SweepPlan> get_gradient(const Circuit &c, int tile_qubits, int amp_bytes, bool reg_f64);
};

// Structure key of a circuit (gate kinds, qubits, which gates are rotations).
void append_structure_key(const Circuit &c, std::vector<int32_t> &key);

// Device-side launch item: one pass of one column over all its tiles.
struct LaunchItem {  // 64 bytes
    uint32_t tile_begin;    // first work-group of this item in the launch
    uint32_t pass;          // index into the pass array
    uint32_t ntiles;
    uint32_t pad;
    uint64_t partial_off;   // in complex doubles
    void *regA;             // lambda
    void *regB;             // phi register 0
    void *regC;             // phi register 1 (blocks of two or four columns)
    void *regD;             // phi registers 2 and 3 (blocks of four columns)
    void *regE;
};

struct ReduceTask {  // 16 bytes: sum partials[off .. off+count) -> results[dest]
    uint64_t off;
    uint32_t count;
    int32_t dest;
};

// Algorithmic flops per amplitude of one inner product of a sweep (one task):
// 8 for <lambda|sigma|phi> (complex conjugate-multiply-add), 6 for the
// rotation adjoint on phi and 6 on lambda, which a block of `width` columns
// shares.
// Algorithmic flops per amplitude per element of a fused pass: the inner
// product (8, or 4 for its real part alone), the rotation adjoint on phi (6)
// and on lambda, shared by the block's columns (6 / width).
inline double sweep_flops_per_amp(int width, bool real_products = false) {
    return (real_products ? 4.0 : 8.0) + 6.0 + 6.0 / width;
}

struct FusedRun {
    int B = 1;                 // columns swept concurrently
    size_t partial_elems = 0;  // complex doubles of partial sums
};

// Blocks run concurrently and scratch sizes for a plan on a register of n qubits.
FusedRun fused_config(const SweepPlan &plan, int requested_streams, size_t state_bytes, size_t free_bytes);

// Arithmetic of a sweep pass over complex64 storage: tiles in FP32 registers
// with each thread's share of an inner product formed in FP32 and summed in
// FP64 beyond the thread (REG_F32), tiles in FP64 registers (REG_F64), or FP32
// registers with every product formed and accumulated in FP64 (REG_F32_EXACT).
// complex128 storage always computes in FP64.
enum RegMode : int { REG_F32 = 0, REG_F64 = 1, REG_F32_EXACT = 2 };

// Kernel launchers (sweep_kernels.hip).
// mats64 / mats32: per gate position 8 values, of which the first two are the
// shear parameters (u, w) of the gate's adjoint (circuit.hpp, adjoint_shear)
// and, for a controlled rotation, the third and fourth its plane rotation
// (c, s) (adjoint_plane), in FP64 and FP32; the kernel reads the table of its
// register precision.
// width: phi registers per item (the plan's column-block width).
// real_products: keep only the real parts of the metric's inner products
// (sweep_kernels_real.hip, or sweep_kernels_real_exact.hip for REG_F32_EXACT;
// the step needs Re G alone).
// ctrl: the plan holds controlled rotations (SweepPlan::ctrl): the kernels with
// the second handler word run.
template <typename R>
void launch_sweep_pass(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                       const DevOp *ops, const DevMap *maps, const double *mats64, const float *mats32,
                       double *partials, int m, int rb, int reg_mode, int width, hipStream_t st,
                       bool real_products = false, bool ctrl = false);
template <typename R>
void launch_sweep_pass_real(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                            const DevOp *ops, const DevMap *maps, const double *mats64, const float *mats32,
                            double *partials, int m, int rb, int reg_mode, int width, hipStream_t st, bool ctrl);
// The REG_F32_EXACT kernels (sweep_kernels_exact.hip: the same source built
// with every product in FP64), complex64 storage only.
void launch_sweep_pass_exact(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                             const DevOp *ops, const DevMap *maps, const float *mats32, double *partials, int m,
                             int rb, int width, hipStream_t st, bool ctrl);
// The REG_F32_EXACT kernels with the real parts of the metric's inner products
// only (sweep_kernels_real_exact.hip).
void launch_sweep_pass_real_exact(const LaunchItem *items, int n_items, uint32_t total_tiles,
                                  const DevPass *passes, const DevOp *ops, const DevMap *maps, const float *mats32,
                                  double *partials, int m, int rb, int width, hipStream_t st, bool ctrl);
void launch_reduce_tasks(const ReduceTask *tasks, int n_tasks, const double *partials, double *results,
                         hipStream_t st);
// The passes without inner products (sweep_kernels_states.hip): lambda and
// the phi registers go through the adjoint gates and the in-pass seeds only.
// width 0: lambda alone (the forward plans: the table then holds the shears
// of the gates themselves, and the kernel applies them).
template <typename R>
void launch_sweep_pass_states(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                              const DevOp *ops, const DevMap *maps, const double *mats64, const float *mats32, int m,
                              int rb, int width, hipStream_t st, bool ctrl = false);


}  // namespace qng
