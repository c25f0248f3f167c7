// batch.hpp -- the metric of many independent ansaetze swept together.
//
// Every ansatz (member) has its own fused sweep plan (sweep.hpp).  The columns
// of all members form one queue (members in increasing register size, columns
// of a member in increasing s, since a member's forward register only moves
// forward).  Columns are admitted into a pool of register pairs until the
// admitted columns cover `target_tiles` work-groups; each launch then runs the
// next pass of every admitted column, whatever member it belongs to, so a
// launch carries tiles of several ansaetze of different size and depth.  A
// column leaves the pool after its last pass and frees its register pair for
// the next column of the queue.  Admission seeds the column: the member's
// forward register advances to y_s, T_s = <y_s|sigma_s|y_s> is taken and the
// pair is set to (y_s, sigma_s y_s) (Sec. 2 recurrences, as in api.cpp).
//
// The schedule depends only on the members' structure and the tuning, not on
// theta: the host builds it once, and the whole metric phase (seeds, sweep
// launches, reductions) can be captured into one hipGraph and replayed with
// new angles (gate matrices are read from device tables).
#pragma once

#include <hip/hip_runtime_api.h>

#include <memory>
#include <vector>

#include "circuit.hpp"
#include "sweep.hpp"

namespace qng {

struct BatchTuning {
    int tile_qubits = 0;        // 0 = library default
    int target_tiles = 4096;    // work-groups per launch the admission aims for
};

struct BatchPrep {              // admission of column block `col` of `member` into a register block
    int member, col;
    uint64_t reg_off;           // byte offset of the block (lambda, then the width phi registers) in the arena
};

struct BatchLaunch {
    uint32_t item_begin, n_items, total_tiles, task_begin, n_tasks, prep_begin, n_preps;
    uint32_t round_begin, n_rounds;   // the launch's column seeds, in rounds
};

// The column seeds before a launch go in rounds: a round holds at most one
// seed per member (a member's seeds depend on each other through its forward
// register), and all of a round's seeds run as one kernel (launch_seed_multi)
// and one reduction of their T.  A seed may first need gates the seed kernel
// does not apply (one kernel per gate, up to fwd_to).
struct BatchSeed {
    int member;
    int fwd_to;                  // gate position the forward register is brought to first, or -1
    int qa, pa, qb, pb;          // rotations the seed kernel applies (qubit, gate position; -1: none)
    int qs, axis, s;             // the seeded column
    uint64_t lam_off, phi_off;   // arena offsets of lambda and the block's top phi register
    uint32_t block_begin, nblocks;   // work-groups within the round (0: seeded on its own, see ctrl)
    int ctrl;                    // 1: rotation s or s - 1 is controlled; the forward register is brought to
                                 // y_s gate by gate and the column seeded with its generator (nblocks 0;
                                 // also 0 for registers below 3 qubits)
};
struct BatchRound {
    uint32_t seed_begin, n_seeds, total_blocks;
    uint32_t n_multi;   // the first n_multi seeds run in the one kernel (registers of >= 3 qubits)
};

struct BatchSchedule {
    int m = 0, rb = 0, amp = 0;
    int width = 1;                                           // columns per lambda sweep (all members)
    bool ctrl = false;                                       // some member has controlled rotations
    std::vector<std::shared_ptr<const SweepPlan>> plans;     // per member
    std::vector<DevPass> passes;                             // merged images
    std::vector<DevOp> ops;
    std::vector<DevMap> maps;
    std::vector<int64_t> gate_base;                          // per member: first row of its matrices
    std::vector<int64_t> lraw_base;                          // per member: first complex of its raw L (P*P),
                                                             // followed by its raw T (P)
    int64_t mat_rows = 0, lraw_elems = 0;
    std::vector<LaunchItem> items;                           // regA/regB: arena offsets
    std::vector<ReduceTask> tasks;
    std::vector<BatchPrep> preps;
    std::vector<BatchSeed> seeds;
    std::vector<BatchRound> rounds;
    std::vector<ReduceTask> seed_tasks;                      // per seed: its T from the round's partials
    std::vector<BatchLaunch> launches;
    std::vector<int> singles;                                // members with P == 1 (no columns)
    uint64_t arena_bytes = 0;
    uint64_t partial_elems = 0;
    int64_t elements = 0;
};

// members: circuits of one register class (same tile width after clamping).
BatchSchedule build_batch_schedule(const std::vector<const Circuit *> &members,
                                   const std::vector<std::shared_ptr<const SweepPlan>> &plans, int amp,
                                   const BatchTuning &tun, uint64_t arena_cap);

// Device images of a schedule (sizes in bytes, 256-aligned sections).
size_t batch_image_bytes(const BatchSchedule &s);

struct BatchDevice {
    char *images = nullptr;            // batch_image_bytes(s)
    char *arena = nullptr;             // s.arena_bytes
    double *fwd_mats = nullptr;        // s.mat_rows x 8 doubles: forward gate matrices
    double *adj_mats = nullptr;        // s.mat_rows x 8 doubles: adjoint gate matrices
    float *adj_mats32 = nullptr;       // the same in FP32
    double *partials = nullptr;        // s.partial_elems complex
    double *lraw = nullptr;            // s.lraw_elems complex
    double *reduce_partials = nullptr; // scratch of the per-primitive reductions
    std::vector<void *> psi;           // per member: forward register (|in> on entry)
    std::vector<double *> traw;        // per member: P complex
};

// Uploads the θ-independent images (passes, ops, maps, items with arena
// pointers, tasks).  Synchronises the stream before returning.
void upload_batch_images(const BatchSchedule &s, const BatchDevice &d, hipStream_t st);

// Enqueues the metric phase of the whole batch: seeds, sweep launches and
// reductions (no host synchronisation, no memsets: capturable).  On return
// (in stream order) member b's forward register holds y_{P_b - 1}.
template <typename R>
void enqueue_batch_metric(const BatchSchedule &s, const std::vector<const Circuit *> &members, const BatchDevice &d,
                          int reg_mode, hipStream_t st, std::vector<hipEvent_t> *events,
                          bool real_products = false);

// Gate position of member b's forward register after the metric phase.
int batch_final_pos(const Circuit &c);

}  // namespace qng
