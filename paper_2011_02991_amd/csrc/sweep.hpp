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
    OP_ROT = 0,      // apply the gate's stored matrix on local bit b0 to both registers
    OP_PRODROT = 1,  // inner product on local bit b0 (axis), then the rotation (same qubit)
    OP_PROD = 2,     // inner product <A|sigma_b0|B> on local bit b0
    OP_CNOT = 3,     // control: local bit b0, or qubit q0 read from the tile base when b0 = 0xFF; target: local b1
    OP_CZ = 4,       // sign (-1)^{x_a x_b}; a: local b0 or base bit q0; b: local b1 or base bit q1
    OP_ZSUM = 5      // Z inner product on qubit q0 outside the tile: +-<A|B>_tile
};

constexpr uint8_t kNoBit = 0xFF;
constexpr int kMaxSlots = 128;      // inner products per pass
constexpr int kMaxTileQubits = 13;

struct DevOp {  // 16 bytes
    uint8_t type, b0, b1, axis;
    uint16_t slot;
    uint8_t q0, q1;
    int32_t gate;   // gate position: row of the matrix table
    int32_t aux;
};

struct DevPass {  // 64 bytes, read with scalar loads
    uint32_t op_begin, n_ops;
    uint16_t n_slots;
    uint8_t m, n, nrest, has_zsum, pad0, pad1;
    uint8_t tile_q[16];
    uint8_t rest_q[32];
};
static_assert(sizeof(DevPass) == 64, "DevPass layout");
static_assert(sizeof(DevOp) == 16, "DevOp layout");

struct HostPass {
    std::vector<uint8_t> tile;          // local bit -> qubit
    std::vector<DevOp> ops;
    std::vector<int32_t> slot_dest;     // per slot: (rotation r) * P + column s
};

struct ColumnPlan {
    int s = 0;                          // rotation index of the column
    std::vector<HostPass> passes;
};

struct SweepPlan {
    int n = 0, m = 0, carriers = 0, P = 0;
    std::vector<ColumnPlan> cols;       // columns 1..P-1 (column 0 has no elements)
    // flattened device images
    std::vector<DevPass> dev_passes;
    std::vector<DevOp> dev_ops;
    std::vector<int64_t> col_pass_begin;   // per column: index of its first pass in dev_passes
    int64_t total_passes = 0, total_ops = 0, max_slots = 0, load_maps = 0;

    size_t device_bytes() const;        // passes + ops (the rest is per call)
    void fill_info(qng_plan_info *out) const;
};

// Build the plan of all columns.  tile_qubits = 0 picks the default for amp_bytes
// (complex64: 12, complex128: 11).
SweepPlan build_sweep_plan(const Circuit &c, int tile_qubits, int amp_bytes, int small);
int default_tile_qubits(int n, int amp_bytes);

struct SweepCache {
    std::map<std::vector<int32_t>, std::shared_ptr<SweepPlan>> plans;
    const SweepPlan &get(const Circuit &c, int tile_qubits, int amp_bytes, int small);
};

// Device-side launch item: one pass of one column over all its tiles.
struct LaunchItem {  // 48 bytes
    uint32_t tile_begin;    // first work-group of this item in the launch
    uint32_t pass;          // index into the pass array
    uint32_t ntiles;
    uint32_t pad;
    uint64_t partial_off;   // in complex doubles
    void *regA;
    void *regB;
    uint64_t pad2;
};

struct ReduceTask {  // 16 bytes: sum partials[off .. off+count) -> results[dest]
    uint64_t off;
    uint32_t count;
    int32_t dest;
};

struct FusedRun {
    int B = 1;                 // columns swept concurrently
    size_t partial_elems = 0;  // complex doubles of partial sums
};

// Columns run concurrently and scratch sizes for a plan on a register of n qubits.
FusedRun fused_config(const SweepPlan &plan, int requested_streams, size_t state_bytes, size_t free_bytes);

// Kernel launchers (sweep_kernels.hip).
template <typename R>
void launch_sweep_pass(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                       const DevOp *ops, const double *mats, double *partials, int max_m, hipStream_t st);
void launch_reduce_tasks(const ReduceTask *tasks, int n_tasks, const double *partials, double *results,
                         hipStream_t st);

}  // namespace qng
