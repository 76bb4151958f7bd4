// Host planner of libpauliprop: gate list -> device schedule.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "pp_device.h"

namespace pp {

struct GateList {
    int n = 0;
    int64_t m = 0;
    std::vector<uint8_t> op;
    std::vector<int32_t> q0, q1, param;
    int32_t n_params = 0;
};

struct DensePass {
    int k = 0;
    uint8_t qubit[8] = {0};
    int op_begin = 0, op_end = 0;
    int64_t ngates = 0;
};

// Dense schedule.  ops are in Heisenberg order (g_m first); maps are built on
// the device from the recipes (gate code and parameter per folded gate).
struct DensePlan {
    bool resident = false;  // whole circuit in one workgroup's LDS
    int k = 0;              // tile qubits (n if resident)
    std::vector<DOp> ops;
    std::vector<int32_t> roff;  // nmaps + 1
    std::vector<uint8_t> rop;
    std::vector<int32_t> rparam;
    std::vector<DensePass> passes;
    int nmaps() const { return (int)roff.size() - 1; }
};

// Sparse schedule: runs of Clifford gates, each closed by one rotation.
struct SparsePlan {
    std::vector<uint32_t> codes;  // Clifford gate codes, Heisenberg order
    std::vector<SparsePassDesc> passes;
};

// compose: fold consecutive single-qubit gates of a wire into one U1 op.
// reorder: let gates on disjoint qubits move past each other when packing
// passes.  Tracked runs disable both, because the term-update count
// U = sum_g |set entering g| depends on the gate order.
// k == n: one resident pass; k < n: passes of k-qubit tiles that always
// contain the lowest `low` qubits.
DensePlan plan_dense(const GateList &g, int k, int low, bool compose, bool reorder);
constexpr int kMaxGroupOps = 16;

// Shape of a GROUP (stored in its header's perm field; 0 = general): a CX
// whose control is the lower (dir 0) or higher (dir 1) digit of the pair,
// then U1 ops on digit sequence code 0 "lower", 1 "higher", 2 "lower,
// higher", 3 "higher, lower": shape = 1 + 4 dir + code.  These eight cover
// most groups of random circuits; the kernels run them as straight-line code.
int group_shape(const DOp *members, int count, int lo);
// Tile size of the register-tile kernel: its passes are ordered into SEG
// segments (see segment_ops in plan.cpp).
constexpr int kSegTileDigits = 6;

// General form: gates [g_begin, g_end) only; forward = g_begin first (the
// adjoint sweep) instead of Heisenberg order; slot (optional, size m): for
// each rotation gate its join slot, stored in DOp::reserved with DOp::b set
// to the rotation's op code.
struct PlanOptions {
    bool compose = true;
    bool group = true;  // pack ops on a common digit pair into GROUP ops
    bool reorder = true;
    bool lookahead = true;  // grow a tile by the gate whose greedy completion of the tile takes the most gates
    // order tiled passes of kSegTileDigits qubits into register segments
    // (SEG headers, which the register-tile kernel needs); the LDS kernels
    // skip SEG headers, so without segments they decode fewer ops
    bool segments = true;
    bool forward = false;
    int64_t g_begin = 0, g_end = -1;
    const std::vector<int32_t> *slot = nullptr;
};
DensePlan plan_dense_opts(const GateList &g, int k, int low, const PlanOptions &o);

// Structural checks of a dense schedule (used by the host-side tests):
// GROUP headers name two distinct digits below k and their members act only
// on them, passes tile the op list, digits are below the tile size, map
// indices are in range.  Returns an empty string or the first violation.
std::string plan_check(const DensePlan &P, int n);

// True when every non-empty tiled pass of kSegTileDigits qubits opens with a
// SEG header (the register-tile kernel can run it).
bool plan_segmented(const DensePlan &P);

// Digit triple (bit mask) the register-tile kernel loads a pass into: the
// first segment's triple when it avoids digits 0 and 1 (lanes then cover 16
// consecutive slots), else digits 3, 4, 5.
uint32_t pass_reg_entry(const DensePlan &P, const DensePass &ps);

// Appends `part` to `all`, offsetting op, map and recipe indices.
void plan_append(DensePlan &all, const DensePlan &part);

// Adjoint-gradient schedule: segments [bounds[s], bounds[s+1]) of the gate
// list; Heisenberg plans per segment (composed) and forward per-gate plans
// per segment; rotation slots in gate order.
struct GradPlan {
    std::vector<int64_t> bounds;
    DensePlan heis, fwd;
    std::vector<int> heis_pass_begin, fwd_pass_begin;  // S + 1 entries each
    std::vector<int32_t> slot_param;                  // slot -> parameter
    std::vector<int32_t> seg_slot_begin;              // S + 1 entries
};
GradPlan plan_gradient(const GateList &g, int k_heis, int k_fwd, int low, int64_t every);
SparsePlan plan_sparse(const GateList &g);

// Clifford frame of a sparse schedule (n <= kFrameMaxN): the rotation axis of
// every pass in the stored frame, and the rows of the linear map from a
// stored key to the x part of its actual string after every Clifford.
struct FramePlan {
    std::vector<FramePassDesc> passes;  // one per sparse pass
    std::vector<uint64_t> xrows;        // n masks over the packed key
};
FramePlan plan_frame(const GateList &g, const SparsePlan &sp);

// structural 3x3 pattern of one gate's Heisenberg map (bit 3*row + col)
unsigned gate_smask(int op);
unsigned smask_compose(unsigned after, unsigned before);

}  // namespace pp
