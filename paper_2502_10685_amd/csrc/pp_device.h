// Internal structures shared by the HIP kernels and the host runtime of
// libpauliprop.  Not part of the public C ABI (include/pauliprop.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pp {

// ---------------------------------------------------------------- dense ops
// Dense layout: the weight of string P(x, z) lives at slot
//   idx = sum_q (x_q << 2q) | (z_q << (2q + 1)),
// i.e. qubit q owns the base-4 digit q (digit value x + 2z: I=0 X=1 Z=2 Y=3).
// This is the paper's index space 0 ... 4^n - 1 (Sec. III-B) with a digit
// order that makes a qubit's four letters one digit of the slot index.
enum : uint8_t { DOP_U1 = 0, DOP_CX = 1, DOP_GROUP = 2, DOP_SEG = 3 };

// One device operation on an LDS tile.  U1: a composed single-qubit map on
// local digit a (a real 3x3 matrix over the X, Y, Z weights, I is fixed).
// CX: control digit a, target digit b.  GROUP: header of the next ngates ops,
// which act only on digits a and b; a thread applies all of them to each
// 16-slot block of those two digits in registers.  SEG: header of the next
// ngates entries (GROUP headers included), whose ops act only on the digit
// triple a < b < smask; the register-tile kernel holds those three digits in
// registers for the whole segment, the LDS kernels skip the header.  16
// bytes, read uniformly.
struct DOp {
    uint8_t kind;
    uint8_t a, b;
    uint8_t ngates;   // gates folded into this op (term-update counting)
    uint16_t smask;   // U1: structural 3x3 pattern, bit (3*row + col)
    uint16_t perm;    // U1: 1 if the map is a signed permutation
    uint32_t map;     // U1: index into the 3x3 map array (9 doubles each)
    uint32_t reserved;
};
static_assert(sizeof(DOp) == 16, "DOp must stay 16 bytes");
// Bit of DOp::perm (any op but SEG): the next op of the pass stays inside
// one wave's quarter of a 6-digit tile as this one does, so 256-thread
// sweeps skip the workgroup barrier between them.
constexpr unsigned kSkipBarrier = 0x8000u;

// A whole circuit run inside one workgroup's LDS (n <= 7).
struct ResidentDesc {
    const void *coef_in;       // start weights (4^n, slot order) or nullptr = the observable
    void *coef_out;            // final weights (4^n, slot order) or nullptr
    uint8_t *pres_out;         // final presence bytes or nullptr
    const DOp *ops;
    const double *maps;
    const uint64_t *obs_x, *obs_z;
    const double *obs_c;
    double *expval_out;
    unsigned long long *counters;  // [0] term updates, [1] final strings
    int32_t nops;
    int32_t n;
    int32_t nterms;
    int32_t reserved;
};

// One pass of one circuit over its 4^(n-k) tiles of 4^k slots.
struct TilePassDesc {
    void *coef;                    // 4^n weights of the circuit
    uint8_t *pres;                 // presence bytes (tracked runs) or nullptr
    const DOp *ops;
    const double *maps;
    unsigned long long *counters;  // [0] term updates (tracked runs)
    int32_t n, k;
    int32_t op_begin, op_end;
    int32_t tile_begin;            // first block of this desc in the launch
    int32_t ntiles;
    uint64_t qubits;               // byte j = global qubit of local digit j (ascending)
    uint32_t reg_entry;            // register-tile kernel: digit triple (bit mask) to load into registers
    uint32_t reserved;
};

// One pass of the adjoint sweep over tiles of 4^k slots (k = n: one tile).
// c: the observable's weights, r: the Pauli coefficients Tr(P rho) of the
// state, both FP64, both propagated forward through the pass's ops.  A U1 op
// of a rotation (b = 3, 4, 5 for RX, RY, RZ) first writes the tile's share of
// its join c^T A r to partials[(reserved - slot_base) * ntiles + tile].
struct GradPassDesc {
    double *c;
    double *r;
    const DOp *ops;
    const double *maps;
    double *partials;
    int32_t n, k;
    int32_t op_begin, op_end;
    int32_t ntiles, slot_base;
    uint64_t qubits;
};

// Block -> descriptor mapping of one tile-pass launch.  Descriptors are
// grouped by tile count (a power of 4); group g covers blocks
// [first_block[g], first_block[g+1]) and block b of it handles tile
// (b - first_block[g]) & ((1 << shift[g]) - 1) of descriptor
// first_desc[g] + ((b - first_block[g]) >> shift[g]).
constexpr int kMaxTileGroups = 8;
struct TileGroups {
    int32_t ngroups;
    int32_t first_block[kMaxTileGroups + 1];
    int32_t first_desc[kMaxTileGroups];
    int32_t shift[kMaxTileGroups];
};

// Start weights and readout of one tiled circuit of a batch: the observable
// is scattered into its 4^n weights, and <O> read out into *out.
struct DenseIODesc {
    void *coef;
    const uint64_t *obs_x, *obs_z;
    const double *obs_c;
    double *out;
    int32_t n, nterms;
};

// Per-circuit composition job: maps[i] = product of the gate matrices of
// recipe entries [roff[i], roff[i+1]) in Heisenberg order.
struct ComposeDesc {
    const int32_t *roff;
    const uint8_t *rop;
    const int32_t *rparam;
    const double *theta;
    double *maps;
    int32_t nmaps;
    int32_t reserved;  // 1: forward maps (each gate's Heisenberg matrix transposed)
};

// --------------------------------------------------------------- sparse ops
// A sparse pass: a run of Clifford gates then (optionally) one rotation.
// Clifford gate code: op | q0 << 8 | q1 << 16 (op in {H, S, CX}).
struct SparsePassDesc {
    int32_t g_begin, g_end;  // range in the Clifford code array
    int32_t rot_op;          // 3..5 for RX/RY/RZ, -1 for none
    int32_t rot_q;
    int32_t rot_param;
    int32_t ngates;          // Cliffords + rotation (term-update counting)
};

// Clifford-frame sparse engine (n <= 31, exact propagation).  The Clifford
// gates are never applied to the strings: the host keeps the accumulated
// Clifford D (processed gates, Heisenberg order) and the stored set S stands
// for D^dag S D.  A rotation exp(-i t sigma/2) on qubit q is then a rotation
// about P = D sigma D^dag in the stored frame (a multi-qubit Pauli with a
// sign), whose child of an anticommuting S is i sin(t) P S.  Keys are packed
// as (z << n) | x.
struct FramePassDesc {
    uint64_t pmask;     // packed key of P's Pauli string
    int32_t sign;       // +1 or -1: P = sign * (the Hermitian Pauli of pmask)
    int32_t a;          // popcount(x & z) of P, mod 4
    int32_t rot_param;  // -1: no rotation (Clifford gates only)
    int32_t ngates;     // gates of the pass (term-update counting)
};

struct FrameBuffers {
    uint64_t *keys;            // list of stored strings: packed keys
    void *coef;                // their weights (FP64 or FP32)
    uint64_t *index;           // hash index, 16-byte slots: [2s] key
                               // (kFrameEmpty when free), [2s + 1] list position
    unsigned long long *cnt;   // pass p reads the list length L and child
                               // count D of pass p - 1 from slot (p-1) mod 3
                               // ([slot] and [3 + slot]), records its own
                               // length in slot p mod 3 and counts its
                               // children in [3 + p mod 3]; [6] overflow
    unsigned long long *updates;
    int64_t cap;               // list capacity
    int64_t slots;             // index slots (power of two, >= 2 cap)
    int32_t slot_bits;
    int32_t n;
};
constexpr uint64_t kFrameEmpty = ~0ull;
constexpr int kFrameMaxN = 31;  // 2n key bits below the empty marker

// ------------------------------------------------------------ launchers
// Dense engine (dense.hip)
// max_maps: the largest nmaps of the descriptors (sizes the grid; any value
// gives the same maps)
hipError_t launch_compose(const ComposeDesc *d_descs, int ndescs, hipStream_t s, int max_maps = 1);
hipError_t launch_resident(const ResidentDesc *d_descs, int ndescs, int n, int dtype_bytes, bool track,
                           hipStream_t s);
hipError_t launch_tile_pass(const TilePassDesc *d_descs, const TileGroups &groups, int k, int dtype_bytes,
                            bool track, hipStream_t s);
// 0: one workgroup per tile; 1: persistent prefetching workgroups (k <= 6)
void set_tile_kernel_variant(int k, int variant);
int tile_kernel_variant(int k);
// threads per workgroup of the untracked LDS-resident kernel for n = 5..7
void set_resident_block(int n, int block);
int resident_block(int n);
hipError_t launch_grad_pass(const GradPassDesc *d_desc, int ntiles, int k, hipStream_t s);
hipError_t launch_grad_init_state(double *r, int n, hipStream_t s);
hipError_t launch_grad_reduce(const double *partials, int nslots, int ntiles, double *rot_grad, hipStream_t s);
hipError_t launch_grad_accumulate(const double *rot_grad, const int32_t *slot_param, int nslots, double *grad,
                                  int nparams, hipStream_t s);
hipError_t launch_copy_f64(const double *src, double *dst, long long count, hipStream_t s);
// count > 1: count weight arrays of 4^n slots back to back (parameter sets)
hipError_t launch_dense_init(void *coef, uint8_t *pres, int n, int dtype_bytes, const uint64_t *x,
                             const uint64_t *z, const double *c, int nterms, hipStream_t s, int count = 1);
hipError_t launch_dense_readout(const void *coef, int n, int dtype_bytes, double *out, hipStream_t s,
                                int count = 1);
// the same for the nd circuits of a batch (one fill, one scatter launch;
// one readout launch), each circuit with the single-circuit arithmetic
hipError_t launch_dense_init_many(const DenseIODesc *d_descs, int nd, int max_n, int dtype_bytes, hipStream_t s);
// rho (2^n x 2^n complex, row-major (re, im) doubles) from the 4^n Pauli
// weights of 2^n rho in slot order; n <= 12
hipError_t launch_density_decode(const void *coef, int n, int dtype_bytes, double *rho, hipStream_t s);
hipError_t launch_dense_readout_many(const DenseIODesc *d_descs, int nd, int dtype_bytes, hipStream_t s);
hipError_t launch_dense_count(const uint8_t *pres, int n, unsigned long long *out, hipStream_t s);
hipError_t launch_dense_compact(const void *coef, const uint8_t *pres, int n, int dtype_bytes, uint64_t *x,
                                uint64_t *z, double *c, unsigned long long *count, int *tile_flags,
                                unsigned long long *tile_vals, int *ticket, hipStream_t s);
size_t resident_lds_bytes(int n, int dtype_bytes, bool track);
constexpr size_t kStaticLdsReserve = 8192;  // op cache + reductions per workgroup
int max_lds_bytes();

// Sparse engine (sparse.hip)
struct SparseBuffers {
    uint64_t *x, *z;      // cap2 entries each
    void *c;
    uint64_t *x2, *z2;    // ping-pong for the sort
    void *c2;
    long long *count;     // [0] live strings, [1] overflow flag, [2] first child,
                          // [3] count before a merge, [4] scan total (8 words)
    long long *scan;      // per-workgroup sums of the multi-workgroup scan (256)
    unsigned long long *updates;
    unsigned int *hist;   // radix histograms (sort_hist_entries(cap2) entries)
    int *tile_flags;      // decoupled look-back state
    unsigned long long *tile_vals;
    int *ticket;
    int64_t cap2;         // capacity of each array (2x the term capacity)
    int64_t max_tiles;
};
hipError_t launch_sparse_init(SparseBuffers &b, int dtype_bytes, const uint64_t *x, const uint64_t *z,
                              const double *c, int nterms, hipStream_t s, double *dropped_total = nullptr);
// Radix-sort shape of the merge, per capacity class (cap2 up to 2^18, up to
// 2^22, larger): 0 = 8 key bits per pass and 8 terms per thread (the
// default), 1 = 8 and 4, 2 = 8 and 16, 3 = 7 and 8, 4 = 7 and 16, 5 = 6 and
// 16.  All shapes give the same order; the histogram array must hold
// sort_hist_entries(cap2) words for any of them.
constexpr int kSortShapeCount = 6;
constexpr int kSortClasses = 3;
int sort_shape_class(long long cap2);
void set_sort_shape(int cls, int shape);
int sort_shape(int cls);
long long sort_hist_entries(long long cap2);
// Truncated propagation (approximate; off when on == 0): a split child with
// more than max_weight non-identity letters is not written, and a merged
// string with more letters or with |weight| < eps is dropped.  The absolute
// weight dropped is summed per tile into dropped[0, tiles) and added, in a
// fixed order, to dropped[max_tiles] (reset by launch_sparse_init).
struct SparseTrunc {
    int32_t on = 0;
    int32_t max_weight = 64;
    double eps = 0.0;
    double *dropped = nullptr;  // max_tiles + 1 doubles
};
hipError_t launch_sparse_pass(SparseBuffers &b, int dtype_bytes, const uint32_t *cliff_codes,
                              const SparsePassDesc &p, const double *theta, hipStream_t s,
                              const SparseTrunc &tr = SparseTrunc{});
hipError_t launch_sparse_merge(SparseBuffers &b, int n, int dtype_bytes, hipStream_t s,
                               const SparseTrunc &tr = SparseTrunc{});
hipError_t launch_sparse_readout(SparseBuffers &b, int dtype_bytes, double *partials, double *out,
                                 hipStream_t s);
// Clifford-frame engine (sparse.hip)
hipError_t launch_frame_init(FrameBuffers &f, int dtype_bytes, const uint64_t *x, const uint64_t *z,
                             const double *c, int nterms, hipStream_t s);
// pass: its index in the schedule (selects the counter slots)
hipError_t launch_frame_pass(FrameBuffers &f, int dtype_bytes, const FramePassDesc &p, const double *theta,
                             int pass, hipStream_t s);
// Strings whose actual form D^dag S D (codes: every Clifford in processing
// order) is made of I and Z only, with their signed weights, into the
// SparseBuffers list out (x = 0, z, weight as FP64), count into out.count[0]
// and the frame's overflow flag into out.count[1].  xrows[j]: mask of the key
// bits whose parity is bit j of the actual x part.
hipError_t launch_frame_x0(FrameBuffers &f, int dtype_bytes, const uint64_t *xrows, const uint32_t *codes,
                           int ncodes, int npasses, SparseBuffers &out, hipStream_t s);
// Every string in its actual form into out (x, z, weight in out's type),
// count and overflow flag into out.count[0], [1].
// The frame's strings after its last pass, in their actual form, into a
// zeroed 4^n DENSE weight array (the ramp of a DENSE evaluation).
hipError_t launch_frame_to_dense(FrameBuffers &f, int dtype_bytes, const uint32_t *codes, int ncodes, int npasses,
                                 void *coef, hipStream_t s);
hipError_t launch_frame_materialize(FrameBuffers &f, int dtype_bytes, const uint32_t *codes, int ncodes,
                                    int npasses, SparseBuffers &out, hipStream_t s);
// list length after `npasses` passes (the counters of the last one)
__host__ __device__ inline int frame_slot_of(int pass) { return ((pass % 3) + 3) % 3; }

}  // namespace pp
