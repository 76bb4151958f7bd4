// Dense (direct-address) engine of libpauliprop.
//
// The weight of every Pauli string lives at a fixed slot of a 4^n array, the
// paper's lambda vector over the index space 0 ... 4^n - 1 (Sec. III-B), so
// strings that coincide after a gate are merged by construction (the reduce()
// of eq. (7) and Examples 3-4 becomes "two contributions land on one slot").
// Slot layout: qubit q owns base-4 digit q, digit value x_q + 2 z_q
// (I=0, X=1, Z=2, Y=3); see pp_device.h.
//
// A device op is either
//   U1: a composed single-qubit map on one digit -- the product, in
//       Heisenberg order, of the 3x3 matrices of every H, S, RX, RY, RZ that
//       acts on that wire between two CX gates touching it (the per-wire
//       composition of Sec. III-C / eq. (5), Table I applied as g^dag P g);
//       the I weight is untouched;
//   CX: the signed swap of the 16 letter pairs of two digits (Sec. III-C:
//       control letter first, XZ <-> -YY).
// A pass streams tiles of 4^k slots (all letters of k qubits, the others
// fixed) through LDS, applies every op of the pass to the tile, and writes
// it back, so HBM sees one read and one write per slot per pass however many
// gates the pass holds.  Circuits with n <= 7 keep all 4^n slots in one
// workgroup's LDS for the whole circuit.
#include <algorithm>
#include <type_traits>

#include "pp_device.h"

namespace pp {

// Bank swizzle for 8-byte LDS words.  The LDS has 64 four-byte banks and
// serves a 64-bit read or write per half-wave, so a half-wave is free of
// conflicts when its 32 slot indices are distinct modulo 32.  With h the
// index bits from bit 5 up, the swizzle XORs bits 0-4 with h << 3, h and
// h >> 2: it is linear over GF(2) and keeps every 32-slot block's set of
// high bits.  With the lane order group_sweep picks per digit pair, every
// digit pair of 5-, 6- and 7-digit tiles is swept without conflicts, and in
// 6-digit tiles so is every pair of digits 0-4 with the lanes drawn from the
// three other digits below 5 alone.
__host__ __device__ constexpr int sw(int i) {
    const int h = i >> 5;
    return i ^ (((h << 3) ^ h ^ (h >> 2)) & 31);
}

// sw(base ^ off) = sw(base) ^ sw(off): slot offsets of an op's letters are
// the same for every lane, so each address costs one XOR with a uniform.

// Workgroup barrier for LDS data: the fences are scoped to LDS, so global
// loads still in flight (a prefetched next tile) are not waited for, which a
// full __syncthreads() would do.  Every barrier in this file orders LDS
// accesses only (threads never exchange data through global memory).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
__device__ __forceinline__ double lds_ld(const T *p, int i) { return (double)p[sw(i)]; }
template <typename T>
__device__ __forceinline__ void lds_st(T *p, int i, double v) { p[sw(i)] = (T)v; }

__device__ __forceinline__ long long morton_slot(uint64_t x, uint64_t z, int n) {
    long long s = 0;
    for (int q = 0; q < n; ++q)
        s |= (long long)(((x >> q) & 1ull) | (((z >> q) & 1ull) << 1)) << (2 * q);
    return s;
}

// slot of the j-th string made of I and Z only (z word = j)
__device__ __forceinline__ long long zonly_slot(long long j, int n) {
    long long s = 0;
    for (int q = 0; q < n; ++q) s |= ((j >> q) & 1ll) << (2 * q + 1);
    return s;
}

// Global slot offset of the local tile index i: local digit j goes to the
// digit of global qubit (qubits >> 8j) & 0xff.  Digits [j0, k) only.
__device__ __forceinline__ long long deposit_digits(int i, uint64_t qubits, int j0, int k) {
    long long g = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j >= j0 && j < k) g |= (long long)((i >> (2 * j)) & 3) << (2 * (int)((qubits >> (8 * j)) & 0xff));
    return g;
}

template <int BLOCK>
__device__ double block_sum_d(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    lds_barrier();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    lds_barrier();
    double tot = 0.0;
    for (int i = 0; i < BLOCK / 64; ++i) tot += red[i];
    return tot;
}

template <int BLOCK>
__device__ long long block_sum_i(long long v, long long *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    lds_barrier();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    lds_barrier();
    long long tot = 0;
    for (int i = 0; i < BLOCK / 64; ++i) tot += red[i];
    return tot;
}

// One row of a U1 map, m0 cx + m1 cy + m2 cz, with its rounding points fixed:
// a product, then two fused multiply-adds.  Every kernel applies maps through
// it, so all of them round alike whatever the surrounding code would let the
// compiler contract (a negation folded in from a CX, say).
__device__ __forceinline__ double map_row(double m0, double m1, double m2, double cx, double cy, double cz) {
    return __builtin_fma(m2, cz, __builtin_fma(m1, cy, m0 * cx));
}

// ----------------------------------------------------------------- U1 op
// Quad u of digit a: the slots base + d * 4^a, d = 0..3, with base the index
// u with a zero digit inserted at position a.  K (tile digits) and BLOCK are
// compile-time, so each thread's quads are loaded together before any store
// (quads are disjoint).  Returns the number of strings created (tracked runs).
template <typename T, bool TRACK, int K, int BLOCK>
__device__ __forceinline__ int u1_apply(T *lc, uint8_t *lp, int a, const double *__restrict__ M, unsigned smask,
                                        int tid) {
    constexpr int NQ = 1 << (2 * (K - 1));
    constexpr int QPT = NQ >= BLOCK ? NQ / BLOCK : 1;
    const int sh = 2 * a;
    const int lowmask = (1 << sh) - 1;
    const double m00 = M[0], m01 = M[1], m02 = M[2];
    const double m10 = M[3], m11 = M[4], m12 = M[5];
    const double m20 = M[6], m21 = M[7], m22 = M[8];
    if (NQ < BLOCK && tid >= NQ) return 0;
    const int oX = sw(1 << sh), oZ = sw(2 << sh), oY = sw(3 << sh);
    // inserting the zero digit and sw are both linear and tid, j * BLOCK
    // have disjoint bits: one per-thread word, the rest uniform
    const int tbase = sw(((tid & ~lowmask) << 2) | (tid & lowmask));
    int iX[QPT], iY[QPT], iZ[QPT];
    double cx[QPT], cy[QPT], cz[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const int uj = j * BLOCK;
        const int sbase = tbase ^ sw(((uj & ~lowmask) << 2) | (uj & lowmask));
        iX[j] = sbase ^ oX;
        iZ[j] = sbase ^ oZ;
        iY[j] = sbase ^ oY;
        cx[j] = (double)lc[iX[j]];
        cy[j] = (double)lc[iY[j]];
        cz[j] = (double)lc[iZ[j]];
    }
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        lc[iX[j]] = (T)map_row(m00, m01, m02, cx[j], cy[j], cz[j]);
        lc[iY[j]] = (T)map_row(m10, m11, m12, cx[j], cy[j], cz[j]);
        lc[iZ[j]] = (T)map_row(m20, m21, m22, cx[j], cy[j], cz[j]);
    }
    int delta = 0;
    if (TRACK) {
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const unsigned old = (unsigned)lp[iX[j]] | ((unsigned)lp[iY[j]] << 1) | ((unsigned)lp[iZ[j]] << 2);
            unsigned nw = 0;
#pragma unroll
            for (int r = 0; r < 3; ++r)
                if ((smask >> (3 * r)) & 7u & old) nw |= 1u << r;
            lp[iX[j]] = (uint8_t)(nw & 1u);
            lp[iY[j]] = (uint8_t)((nw >> 1) & 1u);
            lp[iZ[j]] = (uint8_t)((nw >> 2) & 1u);
            delta += __popc(nw) - __popc(old);
        }
    }
    return delta;
}

// ----------------------------------------------------------------- CX op
// Group u of digits (a = control, b = target): the 16 slots base + dc*4^a +
// dt*4^b.  CX conjugation maps (xc, zc, xt, zt) to (xc, zc^zt, xt^xc, zt)
// with a sign flip iff xc & zt & !(xt ^ zc); the map is an involution, so
// the 12 moving slots form 6 signed swaps.  Work item w = pair * NG + group,
// so every thread gets the same number of swaps.
struct CxPair { int dc1, dt1, dc2, dt2, neg; };
__device__ __forceinline__ CxPair cx_pair(int p) {
    // the six (control digit, target digit) pairs in ascending order of the
    // first slot; digit value x + 2z
    int found = 0;
    CxPair out{0, 0, 0, 0, 0};
#pragma unroll
    for (int dc = 0; dc < 4; ++dc)
#pragma unroll
        for (int dt = 0; dt < 4; ++dt) {
            const int xc = dc & 1, zc = dc >> 1, xt = dt & 1, zt = dt >> 1;
            const int dc2 = xc | ((zc ^ zt) << 1), dt2 = (xt ^ xc) | (zt << 1);
            if (dc2 * 4 + dt2 > dc * 4 + dt) {
                if (found == p) out = CxPair{dc, dt, dc2, dt2, xc & zt & ((xt ^ zc) ^ 1)};
                ++found;
            }
        }
    return out;
}

template <typename T, bool TRACK, int K, int BLOCK>
__device__ __forceinline__ void cx_apply(T *lc, uint8_t *lp, int a, int b, int tid) {
    constexpr int NG = 1 << (2 * (K - 2));
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int mlo = (1 << (2 * lo)) - 1, mhi = (1 << (2 * hi)) - 1;
    const int sa = 2 * a, sb = 2 * b;
    if constexpr (NG >= BLOCK) {
        // one thread per 16-slot group, all six swaps
        int o1[6], o2[6];
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const CxPair pr = cx_pair(p);
            o1[p] = sw((pr.dc1 << sa) | (pr.dt1 << sb));
            o2[p] = sw((pr.dc2 << sa) | (pr.dt2 << sb));
        }
#pragma unroll 1
        for (int j = 0; j < NG / BLOCK; ++j) {
            const int u = tid + j * BLOCK;
            int v = ((u & ~mlo) << 2) | (u & mlo);
            v = ((v & ~mhi) << 2) | (v & mhi);
            const int sv = sw(v);
            double v1[6], v2[6];
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                v1[p] = (double)lc[sv ^ o1[p]];
                v2[p] = (double)lc[sv ^ o2[p]];
            }
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const bool neg = cx_pair(p).neg;
                lc[sv ^ o1[p]] = (T)(neg ? -v2[p] : v2[p]);
                lc[sv ^ o2[p]] = (T)(neg ? -v1[p] : v1[p]);
                if (TRACK) {
                    const uint8_t p1 = lp[sv ^ o1[p]], p2 = lp[sv ^ o2[p]];
                    lp[sv ^ o1[p]] = p2;
                    lp[sv ^ o2[p]] = p1;
                }
            }
        }
    } else {
        // fewer groups than threads: work item w = pair * NG + group
        constexpr int NW = 6 * NG;
        constexpr int WPT = (NW + BLOCK - 1) / BLOCK;
        int i1[WPT], i2[WPT];
        bool neg[WPT], live[WPT];
        double v1[WPT], v2[WPT];
#pragma unroll
        for (int j = 0; j < WPT; ++j) {
            const int w = tid + j * BLOCK;
            live[j] = (NW % BLOCK == 0) || w < NW;
            const int u = w & (NG - 1);
            const CxPair pr = cx_pair(w / NG);
            int v = ((u & ~mlo) << 2) | (u & mlo);
            v = ((v & ~mhi) << 2) | (v & mhi);
            const int sv = sw(v);
            i1[j] = sv ^ sw((pr.dc1 << sa) | (pr.dt1 << sb));
            i2[j] = sv ^ sw((pr.dc2 << sa) | (pr.dt2 << sb));
            neg[j] = pr.neg;
            if (live[j]) {
                v1[j] = (double)lc[i1[j]];
                v2[j] = (double)lc[i2[j]];
            }
        }
#pragma unroll
        for (int j = 0; j < WPT; ++j) {
            if (!live[j]) continue;
            lc[i1[j]] = (T)(neg[j] ? -v2[j] : v2[j]);
            lc[i2[j]] = (T)(neg[j] ? -v1[j] : v1[j]);
            if (TRACK) {
                const uint8_t p1 = lp[i1[j]], p2 = lp[i2[j]];
                lp[i1[j]] = p2;
                lp[i2[j]] = p1;
            }
        }
    }
}

// The six signed swaps of CX as (control digit, target digit) pairs, derived
// at compile time from the rule above; in the paper's letters they are
// (I,Z)<->(Z,Z), (I,Y)<->(Z,Y), (X,I)<->(X,X), (X,Z)<->-(Y,Y), (X,Y)<->(Y,Z),
// (Y,I)<->(Y,X) (digit values I=0 X=1 Z=2 Y=3).
struct CxPairC { int dc1, dt1, dc2, dt2, neg; };
constexpr CxPairC cx_pair_c(int p) {
    int found = 0;
    for (int dc = 0; dc < 4; ++dc)
        for (int dt = 0; dt < 4; ++dt) {
            const int xc = dc & 1, zc = dc >> 1, xt = dt & 1, zt = dt >> 1;
            const int dc2 = xc | ((zc ^ zt) << 1), dt2 = (xt ^ xc) | (zt << 1);
            if (dc2 * 4 + dt2 > dc * 4 + dt) {
                if (found == p) return CxPairC{dc, dt, dc2, dt2, xc & zt & ((xt ^ zc) ^ 1)};
                ++found;
            }
        }
    return CxPairC{0, 0, 0, 0, 0};
}
static_assert(cx_pair_c(3).dc1 == 1 && cx_pair_c(3).dt1 == 2 && cx_pair_c(3).dc2 == 3 && cx_pair_c(3).dt2 == 3 &&
                  cx_pair_c(3).neg == 1,
              "XZ <-> -YY");

template <bool CTRL_LO, int P>
__device__ __forceinline__ void cx_swap(double *v) {
    constexpr CxPairC pr = cx_pair_c(P);
    constexpr int e1 = CTRL_LO ? pr.dc1 + 4 * pr.dt1 : pr.dt1 + 4 * pr.dc1;
    constexpr int e2 = CTRL_LO ? pr.dc2 + 4 * pr.dt2 : pr.dt2 + 4 * pr.dc2;
    const double t1 = v[e1], t2 = v[e2];
    v[e1] = pr.neg ? -t2 : t2;
    v[e2] = pr.neg ? -t1 : t1;
}

// CX on a 16-register block v[dlo + 4 * dhi] of two digits; CTRL_LO: the
// control is the lower digit of the pair.
template <bool CTRL_LO>
__device__ __forceinline__ void cx_regs(double *v) {
    cx_swap<CTRL_LO, 0>(v);
    cx_swap<CTRL_LO, 1>(v);
    cx_swap<CTRL_LO, 2>(v);
    cx_swap<CTRL_LO, 3>(v);
    cx_swap<CTRL_LO, 4>(v);
    cx_swap<CTRL_LO, 5>(v);
}

template <bool LO, int Q>
__device__ __forceinline__ void u1_quad(double *v, const double (&m)[9]) {
    constexpr int iX = LO ? 1 + 4 * Q : Q + 4, iZ = LO ? 2 + 4 * Q : Q + 8, iY = LO ? 3 + 4 * Q : Q + 12;
    const double cx = v[iX], cy = v[iY], cz = v[iZ];
    v[iX] = map_row(m[0], m[1], m[2], cx, cy, cz);
    v[iY] = map_row(m[3], m[4], m[5], cx, cy, cz);
    v[iZ] = map_row(m[6], m[7], m[8], cx, cy, cz);
}

// U1 (3x3 map M over X, Y, Z) on one digit of a 16-register block; LO: the
// lower digit of the pair.
template <bool LO>
__device__ __forceinline__ void u1_regs_m(double *v, const double (&m)[9]) {
    u1_quad<LO, 0>(v, m);
    u1_quad<LO, 1>(v, m);
    u1_quad<LO, 2>(v, m);
    u1_quad<LO, 3>(v, m);
}

// Ops and their maps are staged through LDS in chunks: one cooperative load
// per chunk instead of a dependent global load per op.
constexpr int OPCH = 32;
template <int CH>
struct OpCacheN {
    DOp ops[CH];
    double maps[CH][9];
};
using OpCache = OpCacheN<OPCH>;

// Stages ops [o0, o0 + cn) and the maps of their U1 ops into an op cache.
// Group sweeps read the maps by scalar loads from global memory instead;
// the copy serves the per-op U1 path (tracked runs) and, for the sweeps,
// brings the maps into L2 before their scalar loads (without it the
// streaming kernel is 5 % slower).
// Ops move as raw 16-byte words from the global address space: copied as a
// struct of bytes they would go through scratch, whose wait covers every
// outstanding vector load (tile prefetches included).
template <int CH>
__device__ __forceinline__ void stage_ops(OpCacheN<CH> *oc, const DOp *ops, const double *maps, int o0, int cn, int tid,
                                          int nthreads) {
    typedef unsigned U4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) U4 *GOps;
    typedef const __attribute__((address_space(1))) double *GMaps;
    for (int j = tid; j < cn; j += nthreads) {
        const U4 w = ((GOps)ops)[o0 + j];
        reinterpret_cast<U4 *>(oc->ops)[j] = w;
        if ((w.x & 0xffu) == DOP_U1) {
            const GMaps src = (GMaps)maps + 9ull * w.z;
#pragma unroll
            for (int k = 0; k < 9; ++k) oc->maps[j][k] = src[k];
        }
    }
}

// Lane order of a group sweep on digits (A, B) of a 4^K-slot tile: thread u
// owns the 16-slot block whose other digits are u's bits deposited at
// pos[0..2(K-2)).  The first five positions are the first five free index
// bits (in lexicographic order of their positions) whose images under sw
// are independent modulo 32, so the 32 lanes of a half-wave hit 32
// distinct bank pairs; the other free bits follow in ascending order.  In a
// 6-digit tile a pair of digits below 5 draws the lanes from the other
// digits below 5 only, so u's bits 6 and 7 (the wave of a 256-thread sweep)
// are digit 5: each wave then reads and writes only the quarter of the tile
// whose digit 5 is its index.
struct LaneOrder {
    int pos[14];
    bool conflict_free;  // the first five positions were found
};
constexpr int gf2_rank(int *v, int n) {
    int r = 0;
    for (int bit = 0; bit < 5; ++bit) {
        int piv = -1;
        for (int i = r; i < n; ++i)
            if ((v[i] >> bit) & 1) {
                piv = i;
                break;
            }
        if (piv < 0) continue;
        const int t = v[r];
        v[r] = v[piv];
        v[piv] = t;
        for (int i = 0; i < n; ++i)
            if (i != r && ((v[i] >> bit) & 1)) v[i] ^= v[r];
        ++r;
    }
    return r;
}
template <int K, int A, int B>
constexpr LaneOrder lane_order() {
    int fr[14] = {0};
    int nf = 0;
    for (int d = 0; d < K; ++d)
        if (d != A && d != B) {
            fr[nf++] = 2 * d;
            fr[nf++] = 2 * d + 1;
        }
    LaneOrder o{};
    for (int j = 0; j < nf; ++j) o.pos[j] = fr[j];
    if (nf < 5) return o;
    // digit 5's two bits come last in fr when the pair avoids it
    const int ns = (K == 6 && B < 5) ? nf - 2 : nf;
    for (int i0 = 0; i0 < ns; ++i0)
        for (int i1 = i0 + 1; i1 < ns; ++i1)
            for (int i2 = i1 + 1; i2 < ns; ++i2)
                for (int i3 = i2 + 1; i3 < ns; ++i3)
                    for (int i4 = i3 + 1; i4 < ns; ++i4) {
                        const int idx[5] = {i0, i1, i2, i3, i4};
                        int c[5] = {0};
                        for (int k = 0; k < 5; ++k) c[k] = sw(1 << fr[idx[k]]) & 31;
                        if (gf2_rank(c, 5) < 5) continue;
                        int j = 0;
                        for (int k = 0; k < 5; ++k) o.pos[j++] = fr[idx[k]];
                        for (int f = 0; f < nf; ++f)
                            if (f != i0 && f != i1 && f != i2 && f != i3 && f != i4) o.pos[j++] = fr[f];
                        o.conflict_free = true;
                        return o;
                    }
    return o;
}

// A 3x3 map into SGPRs by scalar loads (the map array is read-only).
typedef const __attribute__((address_space(4))) double *ConstMaps;
__device__ __forceinline__ void load_map(double (&m)[9], ConstMaps src) {
#pragma unroll
    for (int q = 0; q < 9; ++q) m[q] = src[q];
}

// The eight common GROUP shapes (see the planner's group_shape): the CX,
// then the U1 ops in order, with the first U1's map m1 already loaded and
// the second's at s2.  The second map is loaded once the first is applied,
// so only one map occupies SGPRs at a time (two would push the kernel past
// its SGPR budget and spill).
template <bool CTRL_LO, int CODE>
__device__ __forceinline__ void shape_apply(double *v, const double (&m1)[9], ConstMaps s2) {
    cx_regs<CTRL_LO>(v);
    u1_regs_m<CODE == 0 || CODE == 2>(v, m1);
    if constexpr (CODE >= 2) {
        double m[9];
        load_map(m, s2);
        u1_regs_m<CODE == 3>(v, m);
    }
}

// A GROUP of cnt ops on digits A < B: each thread owns whole 16-slot blocks
// (all letters of the two digits), applies every member op in registers and
// writes the block back once.  Compiled per digit pair, so the sixteen
// letter offsets are constants.  A group of one of the eight common shapes
// (shape != 0) runs as straight-line code: the CX renames registers instead
// of moving them, both maps are loaded at once, and each shape writes the
// block back from its own registers; the same operations in the same order
// as the general member loop, so the same results.
template <typename T, int K, int BLOCK, int A, int B>
__device__ __forceinline__ void group_sweep(T *lc, const DOp *ops, int first, int cnt, int tid, const DOp *gops,
                                            const double *gmaps, int shape, uint32_t map1, uint32_t map2) {
    constexpr int NG = 1 << (2 * (K - 2));
    constexpr int GPT = NG >= BLOCK ? NG / BLOCK : 1;
    constexpr LaneOrder lo = lane_order<K, A, B>();
    static_assert(K < 5 || lo.conflict_free, "every digit pair of a 5- to 7-digit tile has a conflict-free lane order");
    static_assert(K != 6 || B == 5 || (lo.pos[6] == 10 && lo.pos[7] == 11), "waves split 6-digit tiles by digit 5");
    if (NG < BLOCK && tid >= NG) return;
#pragma unroll 1
    for (int j = 0; j < GPT; ++j) {
        int u = tid + j * BLOCK;
        // the addresses below are loop invariant for every digit pair; an
        // opaque u keeps the compiler from hoisting all pairs' addresses out
        // of the tile loop (they would not fit in registers)
        __asm__ volatile("" : "+v"(u));
        int v0 = 0;
#pragma unroll
        for (int q = 0; q < 2 * (K - 2); ++q) v0 |= ((u >> q) & 1) << lo.pos[q];
        const int sv = sw(v0);
        // word 0 of member t sits in lane t (cnt <= kMaxGroupOps < 64): one LDS
        // read issued with the block's reads instead of a round trip per
        // member.  Only when every lane of the wave takes part (NG >= 64);
        // smaller tiles read each member's word on its own.
        const int lane = tid & 63;
        uint32_t wl = 0, ml = 0;  // word 0 and map index of member `lane`
        if constexpr (NG >= 64) {
            if (shape == 0) {  // a shape's fields all came with its header
                const uint32_t *ow = reinterpret_cast<const uint32_t *>(&ops[first + (lane < cnt ? lane : 0)]);
                wl = ow[0];
                ml = ow[2];
            }
        }
        // Slot sv ^ c of the block, with c = cl | ch (cl the bits below 5,
        // ch the rest, which sv does not have): the tile starts on a 256-byte
        // boundary of LDS (every kernel aligns its dynamic LDS so), so its
        // byte address is ((base + sv * size) ^ cl * size) + ch * size, one
        // XOR per slot with ch * size in the instruction's offset field.
        typedef __attribute__((address_space(3))) T LT;
        const unsigned svb = (unsigned)(size_t)(LT *)lc + (unsigned)sv * (unsigned)sizeof(T);
        auto slot = [&](int e) -> LT & {
            const int c = sw(((e & 3) << (2 * A)) | ((e >> 2) << (2 * B)));
            return *(LT *)(size_t)((svb ^ (unsigned)((c & 31) * (int)sizeof(T))) + (unsigned)((c & ~31) * (int)sizeof(T)));
        };
        constexpr bool kShapes = NG >= 64;
        // a shape's first map: its index came with the header, so its
        // scalar loads go out before the block's LDS reads
        double m1[9];
        if (kShapes && shape != 0) load_map(m1, (ConstMaps)gmaps + 9ull * map1);
        double v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = (double)slot(e);
        if constexpr (kShapes) {
            if (shape != 0) {
                const ConstMaps s2 = (ConstMaps)gmaps + 9ull * map2;
#define PP_SHAPE_CASE(S_, LO_, CODE_)                                                                          \
    case S_:                                                                                                   \
        shape_apply<LO_, CODE_>(v, m1, s2);                                                                    \
        _Pragma("unroll") for (int e = 0; e < 16; ++e) slot(e) = (T)v[e];                                      \
        continue;
                switch (shape) {
                    PP_SHAPE_CASE(1, true, 0)
                    PP_SHAPE_CASE(2, true, 1)
                    PP_SHAPE_CASE(3, true, 2)
                    PP_SHAPE_CASE(4, true, 3)
                    PP_SHAPE_CASE(5, false, 0)
                    PP_SHAPE_CASE(6, false, 1)
                    PP_SHAPE_CASE(7, false, 2)
                    PP_SHAPE_CASE(8, false, 3)
                default: break;
                }
#undef PP_SHAPE_CASE
            }
        }
#pragma unroll 1
        for (int t = 0; t < cnt; ++t) {
            const uint32_t w0 = NG >= 64
                                    ? __builtin_amdgcn_readlane(wl, t)
                                    : __builtin_amdgcn_readfirstlane(reinterpret_cast<const uint32_t *>(&ops[first + t])[0]);
            const int kind = w0 & 0xff, da = (w0 >> 8) & 0xff;
            if (kind == DOP_U1) {
                // the map (the same for every lane) comes into SGPRs by
                // scalar loads from the global map array (gops: the group's
                // ops in global memory, gmaps: the map array, both
                // wave-uniform) and is the FMAs' scalar operand: nine fewer
                // LDS reads and about 16 fewer VGPRs than an LDS copy, which
                // lets the 6-qubit streaming kernel run four waves per SIMD
                typedef const __attribute__((address_space(4))) uint32_t *CW;
                typedef const __attribute__((address_space(4))) double *CD;
                // the map index from the lane-indexed op words (no dependent
                // scalar load before the map's own)
                const uint32_t mi = NG >= 64 ? (uint32_t)__builtin_amdgcn_readlane(ml, t)
                                             : ((CW)(gops + first + t))[2];
                const CD src = (CD)gmaps + 9ull * mi;
                double m[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) m[q] = src[q];
                if (da == A) u1_regs_m<true>(v, m);
                else u1_regs_m<false>(v, m);
            } else {
                if (da == A) cx_regs<true>(v);
                else cx_regs<false>(v);
            }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) slot(e) = (T)v[e];
    }
}

template <typename T, int K, int BLOCK>
__device__ __forceinline__ void group_apply(T *lc, int a, int b, const DOp *ops, int first, int cnt, int tid,
                                            const DOp *gops, const double *gmaps, int shape, uint32_t map1 = 0,
                                            uint32_t map2 = 0) {
#define PP_GROUP_CASE(A_, B_)                                                                                       \
    case (A_) * 8 + (B_):                                                                                          \
        if constexpr ((B_) < K)                                                                                    \
            group_sweep<T, K, BLOCK, (A_), (B_)>(lc, ops, first, cnt, tid, gops, gmaps, shape, map1, map2);        \
        return;
    if constexpr (K <= 6) {  // only the pairs that exist: a shallower branch tree
        switch (a * 8 + b) {
            PP_GROUP_CASE(0, 1) PP_GROUP_CASE(0, 2) PP_GROUP_CASE(0, 3) PP_GROUP_CASE(0, 4) PP_GROUP_CASE(0, 5)
            PP_GROUP_CASE(1, 2) PP_GROUP_CASE(1, 3) PP_GROUP_CASE(1, 4) PP_GROUP_CASE(1, 5)
            PP_GROUP_CASE(2, 3) PP_GROUP_CASE(2, 4) PP_GROUP_CASE(2, 5)
            PP_GROUP_CASE(3, 4) PP_GROUP_CASE(3, 5) PP_GROUP_CASE(4, 5)
        default: return;  // the planner emits GROUP headers with a < b < K only
        }
    } else {
        switch (a * 8 + b) {
            PP_GROUP_CASE(0, 1) PP_GROUP_CASE(0, 2) PP_GROUP_CASE(0, 3) PP_GROUP_CASE(0, 4) PP_GROUP_CASE(0, 5)
            PP_GROUP_CASE(0, 6) PP_GROUP_CASE(1, 2) PP_GROUP_CASE(1, 3) PP_GROUP_CASE(1, 4) PP_GROUP_CASE(1, 5)
            PP_GROUP_CASE(1, 6) PP_GROUP_CASE(2, 3) PP_GROUP_CASE(2, 4) PP_GROUP_CASE(2, 5) PP_GROUP_CASE(2, 6)
            PP_GROUP_CASE(3, 4) PP_GROUP_CASE(3, 5) PP_GROUP_CASE(3, 6) PP_GROUP_CASE(4, 5) PP_GROUP_CASE(4, 6)
            PP_GROUP_CASE(5, 6)
        default: return;  // the planner emits GROUP headers with a < b < K only
        }
    }
#undef PP_GROUP_CASE
}

// Applies ops [o0, o1) to an LDS tile of 4^K slots.  For tracked runs it
// accumulates term updates: every op adds ngates * (strings in the tile
// before it), and U1 ops that can create strings update that count.
// A 64-bit value made wave-uniform.  readfirstlane returns a signed int:
// each half is widened through uint32_t, or a low half with bit 31 set
// would fill the high half with ones.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Untracked 256-thread sweeps of a 6-digit tile: an op on digits below 5
// reads and writes only the quarter of the tile that belongs to the
// sweeping thread's wave (digit 5 = wave index, see lane_order), so between
// two such ops no workgroup barrier is needed.  The planner marks each op
// after which the barrier can go (kSkipBarrier in its perm field; it moves
// the pass's cheapest digit to position 5 first).  The LDS completes a
// wave's instructions in issue order, and fences at wavefront scope keep
// the compiler from moving the next op's accesses above this op's.
template <int K, int BLOCK, bool TRACK>
constexpr bool kWaveSplit = K == 6 && BLOCK == 256 && !TRACK;

__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <typename T, bool TRACK, int K, int BLOCK, int CH = OPCH>
__device__ __forceinline__ void run_ops(T *lc, uint8_t *lp, const DOp *__restrict__ ops, const double *__restrict__ maps, int o0,
                        int o1, long long &tcount, long long &updates, long long *redi, OpCacheN<CH> *oc,
                        bool preloaded = false) {
    const int tid = threadIdx.x;
    const double *gmaps = (const double *)uniform_u64((uint64_t)maps);
    const DOp *gops0 = (const DOp *)uniform_u64((uint64_t)ops);
    int cb = o0;
    while (cb < o1) {
        const int cn = (o1 - cb) < CH ? (o1 - cb) : CH;
        const DOp *gops = gops0 + cb;  // gops[i] is oc->ops[i]
        lds_barrier();
        if (!preloaded) {
            stage_ops<CH>(oc, ops, maps, cb, cn, tid, BLOCK);
            lds_barrier();
        }
        preloaded = false;
        // the next op's header (16 bytes) is read from LDS while the
        // current op runs, so decoding an op waits for no LDS round trip
        typedef unsigned HdrW __attribute__((ext_vector_type(4)));
        HdrW hdr = reinterpret_cast<const HdrW *>(&oc->ops[0])[0];
        int i = 0;
        while (i < cn) {
            // op fields are the same for every lane: keep them in SGPRs
            const uint32_t w0 = __builtin_amdgcn_readfirstlane(hdr.x);
            const uint32_t w1 = __builtin_amdgcn_readfirstlane(hdr.y);
            const uint32_t w2 = __builtin_amdgcn_readfirstlane(hdr.z);
            const uint32_t w3 = __builtin_amdgcn_readfirstlane(hdr.w);
            const int kind = w0 & 0xff, a = (w0 >> 8) & 0xff, b = (w0 >> 16) & 0xff, ngates = (w0 >> 24) & 0xff;
            const unsigned smask = w1 & 0xffff, perm = (w1 >> 16) & ~kSkipBarrier;
            const bool skip_barrier = kWaveSplit<K, BLOCK, TRACK> && ((w1 >> 16) & kSkipBarrier);
            {
                const int nxt = i + 1 + (kind == DOP_GROUP ? ngates : 0);
                if (nxt < cn) hdr = reinterpret_cast<const HdrW *>(&oc->ops[nxt])[0];
            }
            if (kind == DOP_SEG) {  // register-tile layout hint: nothing to do in LDS
                ++i;
                continue;
            }
            if (kind == DOP_GROUP) {
                if (i + 1 + ngates > cn) break;  // reload the chunk from this header
                if constexpr (K >= 2)
                    group_apply<T, K, BLOCK>(lc, a, b, oc->ops, i + 1, ngates, tid, gops, gmaps, (int)perm, w2, w3);
                i += 1 + ngates;
            } else if (!TRACK && K >= 2 && K <= 7) {
                // untracked U1 or CX alone: a group sweep of one op over its
                // digit pair (a U1 borrows a neighbouring digit), which keeps
                // the conflict-free lane order of the pair
                const int other = kind == DOP_U1 ? (a == 0 ? 1 : a - 1) : b;
                if constexpr (K >= 2)
                    group_apply<T, K, BLOCK>(lc, a < other ? a : other, a < other ? other : a, oc->ops, i, 1, tid, gops,
                                             gmaps, 0);
                ++i;
            } else if (kind == DOP_U1) {
                const int delta = u1_apply<T, TRACK, K, BLOCK>(lc, lp, a, oc->maps[i], smask, tid);
                if (TRACK) {
                    updates += tcount * ngates;
                    if (!perm) tcount += block_sum_i<BLOCK>(delta, redi);
                }
                ++i;
            } else {
                if constexpr (K >= 2) cx_apply<T, TRACK, K, BLOCK>(lc, lp, a, b, tid);
                if (TRACK) updates += tcount * ngates;
                ++i;
            }
            if (skip_barrier) wave_lds_order();
            else lds_barrier();
        }
        cb += i;
    }
}

// ------------------------------------------------------- resident kernel
// One workgroup runs one whole circuit (n <= 7) in LDS: builds the
// observable, applies every op, reads out <O> and optionally stores the
// final weights / presence for pp_get_terms.
template <typename T, bool TRACK, int N, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu((N >= 7 && BLOCK <= 256) ? 2 : (BLOCK >= 1024 ? 4 : (BLOCK >= 512 ? 2 : 4))))) void resident_kernel(const ResidentDesc *__restrict__ descs) {
    extern __shared__ __align__(256) unsigned char smem[];
    __shared__ double redd[BLOCK / 64];
    __shared__ long long redi[BLOCK / 64];
    __shared__ OpCache oc;
    const ResidentDesc d = descs[blockIdx.x];
    constexpr int n = N;
    constexpr int size = 1 << (2 * N);
    T *lc = reinterpret_cast<T *>(smem);
    uint8_t *lp = smem + (size_t)size * sizeof(T);
    const int tid = threadIdx.x;

    for (int i = tid; i < size; i += BLOCK) {
        lc[i] = (T)0;
        if (TRACK) lp[i] = 0;
    }
    lds_barrier();
    if (d.coef_in) {
        const T *in = reinterpret_cast<const T *>(d.coef_in);
        for (int i = tid; i < size; i += BLOCK) lc[sw(i)] = in[i];
    } else if (tid == 0) {
        for (int t = 0; t < d.nterms; ++t) {
            const int s = (int)morton_slot(d.obs_x[t], d.obs_z[t], n);
            lc[sw(s)] = (T)((double)lc[sw(s)] + d.obs_c[t]);
            if (TRACK) lp[sw(s)] = 1;
        }
    }
    lds_barrier();

    long long tcount = 0, updates = 0;
    if (TRACK) {
        long long mine = 0;
        for (int i = tid; i < size; i += BLOCK) mine += lp[i];
        tcount = block_sum_i<BLOCK>(mine, redi);
    }
    run_ops<T, TRACK, N, BLOCK>(lc, lp, d.ops, d.maps, 0, d.nops, tcount, updates, redi, &oc);

    double part = 0.0;
    for (int j = tid; j < (1 << n); j += BLOCK) part += lds_ld(lc, (int)zonly_slot(j, n));
    const double total = block_sum_d<BLOCK>(part, redd);
    if (tid == 0) {
        *d.expval_out = total;
        if (TRACK && d.counters) {
            d.counters[0] = (unsigned long long)updates;
            d.counters[1] = (unsigned long long)tcount;
        }
    }
    if (d.coef_out) {
        T *out = reinterpret_cast<T *>(d.coef_out);
        for (int i = tid; i < size; i += BLOCK) out[i] = lc[sw(i)];
    }
    if (TRACK && d.pres_out) {
        for (int i = tid; i < size; i += BLOCK) d.pres_out[i] = lp[sw(i)];
    }
}

// ------------------------------------------------------------ tile kernel
// Block -> (desc, tile).  The tile's slots are the 4^k combinations of the
// pass's k qubits with the other n-k digits fixed to the tile index.  Local
// digit j is global qubit qubit[j] (ascending), so the leading local digits
// that equal their qubit form contiguous runs in HBM.
template <typename T, bool TRACK, int K, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu((BLOCK == 64 && K >= 6) ? 1 : (K >= 7 ? 2 : 4)))) void tile_kernel(const TilePassDesc *__restrict__ descs, TileGroups grp) {
    extern __shared__ __align__(256) unsigned char smem[];
    __shared__ long long redi[BLOCK / 64];
    __shared__ OpCache oc;
    const int b = blockIdx.x;
    int gi0 = 0;
    while (gi0 + 1 < grp.ngroups && b >= grp.first_block[gi0 + 1]) ++gi0;
    const int rel = b - grp.first_block[gi0];
    const TilePassDesc d = descs[grp.first_desc[gi0] + (rel >> grp.shift[gi0])];
    const long long tile = rel & ((1 << grp.shift[gi0]) - 1);
    constexpr int k = K;
    const int n = d.n;
    constexpr int size = 1 << (2 * K);
    T *lc = reinterpret_cast<T *>(smem);
    uint8_t *lp = smem + (size_t)size * sizeof(T);
    const int tid = threadIdx.x;

    unsigned inmask = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < k) inmask |= 1u << (unsigned)((d.qubits >> (8 * j)) & 0xff);
    long long base = 0;
    {
        long long t = tile;
        for (int q = 0; q < n; ++q) {
            if ((inmask >> q) & 1u) continue;
            base |= (t & 3ll) << (2 * q);
            t >>= 2;
        }
    }
    // local index i = tid + r * BLOCK with BLOCK a power of two: tid and
    // r * BLOCK have disjoint bits, so their digit deposits simply OR, and
    // the r part is the same for every lane
    static_assert((BLOCK & (BLOCK - 1)) == 0 && BLOCK <= size, "a tile holds at least one slot per thread");
    const long long toff = base | deposit_digits(tid, d.qubits, 0, k);

    T *g = reinterpret_cast<T *>(d.coef);
    const int stid = sw(tid);  // sw(tid + r * BLOCK) = sw(tid) ^ sw(r * BLOCK)
    for (int i = tid, r = 0; i < size; i += BLOCK, ++r) {
        const long long gi = toff | deposit_digits(r * BLOCK, d.qubits, 0, k);
        const int li = stid ^ sw(r * BLOCK);
        lc[li] = g[gi];
        if (TRACK) lp[li] = d.pres[gi];
    }
    lds_barrier();

    long long tcount = 0, updates = 0;
    if (TRACK) {
        long long mine = 0;
        for (int i = tid; i < size; i += BLOCK) mine += lp[i];
        tcount = block_sum_i<BLOCK>(mine, redi);
    }
    run_ops<T, TRACK, K, BLOCK>(lc, lp, d.ops, d.maps, d.op_begin, d.op_end, tcount, updates, redi, &oc);

    for (int i = tid, r = 0; i < size; i += BLOCK, ++r) {
        const long long gi = toff | deposit_digits(r * BLOCK, d.qubits, 0, k);
        const int li = stid ^ sw(r * BLOCK);
        g[gi] = lc[li];
        if (TRACK) d.pres[gi] = lp[li];
    }
    if (TRACK && tid == 0 && updates) atomicAdd(d.counters, (unsigned long long)updates);
}

// Weights are read and written with buffer instructions: one resource per
// tile (base = the tile's first slot), the lane's slot offset in a VGPR and
// the register's in an SGPR, so the 64 accesses of a lane need no address
// registers.  Both offsets are below 2^31 bytes when the tile's qubits are
// all below 14 (the launcher only picks this kernel for n <= 14).  Every
// weight is read once and written once per pass, so both carry the
// non-temporal hint (nt): the streamed array then does not push the op
// lists and maps, which every tile re-reads, out of L2.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, -1, 0x00020000);
}
// cache-policy operand of the buffer builtins: bit 1 is nt on gfx950
constexpr int kNonTemporal = 2;
template <typename T>
struct BufIO;
template <>
struct BufIO<double> {
    typedef unsigned V __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, kNonTemporal));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, double v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, vo, so, kNonTemporal);
    }
};
template <>
struct BufIO<float> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, kNonTemporal));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, kNonTemporal);
    }
};

// ------------------------------------------------- streaming tile kernel
// Persistent form of tile_kernel for untracked runs: a co-resident grid
// walks the launch's tiles with stride gridDim.x, and every workgroup issues
// the global loads of its next tile into registers before it runs the ops of
// the current one, so HBM latency overlaps the LDS work (the barriers in
// run_ops are LDS-scoped and do not wait for those loads).  Weights move
// with buffer instructions: the tile base is uniform, the thread's slot
// offset (digits 0-3) is one VGPR and the register's offset (digits 4 and
// up) is uniform, so the prefetch costs no address registers; the launcher
// takes this kernel only for n <= 14, where both offsets fit 31 bits.
struct TileLoc {
    const TilePassDesc *d;
    long long base;
    unsigned voff;  // bytes
};

template <typename T, int K, int BLOCK>
__device__ __forceinline__ TileLoc locate_tile(const TilePassDesc *__restrict__ descs, const TileGroups &grp, int b,
                                               int tid) {
    int g = 0;
    while (g + 1 < grp.ngroups && b >= grp.first_block[g + 1]) ++g;
    const int rel = b - grp.first_block[g];
    const TilePassDesc *d = descs + grp.first_desc[g] + (rel >> grp.shift[g]);
    const long long tile = rel & ((1 << grp.shift[g]) - 1);
    const uint64_t qubits = d->qubits;
    const int n = d->n;
    unsigned inmask = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < K) inmask |= 1u << (unsigned)((qubits >> (8 * j)) & 0xff);
    // the tile index's digits go to the qubits outside the tile, lowest
    // first: one step per outside qubit
    long long base = 0, t = tile;
    unsigned out = ~inmask & ((1u << n) - 1u);
    while (out) {
        const int q = __builtin_ctz(out);
        out &= out - 1u;
        base |= (t & 3ll) << (2 * q);
        t >>= 2;
    }
    // the thread index supplies the low bits of the slot index (digits 0-3,
    // and the low bit of digit 4 for 512 threads); deposits of disjoint bits
    // OR.  In 32 bits (the offset is below 2^31 bytes): 64-bit digit values
    // would be hoisted out of the tile loop and spilled.
    unsigned voff = 0;
#pragma unroll
    for (int j = 0; j < (BLOCK > 256 ? 5 : 4); ++j)
        voff |= (((unsigned)tid >> (2 * j)) & 3u) << (2 * (unsigned)((qubits >> (8 * j)) & 0xff));
    return TileLoc{d, base, voff * (unsigned)sizeof(T)};
}

// Byte offset (uniform) of row r of a thread's slots: the row supplies the
// tile digits from 4 up; in 32 bits, with each digit value times the
// element size a constant, so a row costs a shift per digit and an OR.
template <typename T, int K, int BLOCK>
__device__ __forceinline__ unsigned stream_soff(uint64_t qubits, int r) {
    unsigned g = 0;
#pragma unroll
    for (int j = 4; j < K; ++j)
        g |= ((((unsigned)(r * BLOCK) >> (2 * j)) & 3u) * (unsigned)sizeof(T)) << (2u * (unsigned)((qubits >> (8 * j)) & 0xff));
    return g;
}

// 256 threads for tiles up to 4^6 slots (four workgroups per CU: at most 128
// VGPRs, and 4 x 37 KiB of LDS in FP64); 512 threads and one workgroup per
// CU for 4^7 slots (its LDS tile is 128 KiB in FP64)
template <int K>
constexpr int kStreamBlock = K >= 7 ? 512 : 256;
template <int K>
constexpr int kStreamWaves = K >= 7 ? 2 : 4;

// ops held per workgroup: every 6-qubit pass of the planner fits (its passes
// have at most 64 op entries); longer passes reload chunks inside run_ops
constexpr int kStreamOps = 64;

template <typename T, int K>
__global__ __launch_bounds__(kStreamBlock<K>) __attribute__((amdgpu_waves_per_eu(kStreamWaves<K>)))
void tile_stream_kernel(const TilePassDesc *__restrict__ descs, TileGroups grp) {
    constexpr int BLOCK = kStreamBlock<K>;
    constexpr int size = 1 << (2 * K);
    constexpr int PER = size / BLOCK;
    static_assert(K >= 4, "the thread index supplies four digits");
    extern __shared__ __align__(256) unsigned char smem[];
    __shared__ long long redi[BLOCK / 64];
    __shared__ OpCacheN<kStreamOps> oc;
    T *lc = reinterpret_cast<T *>(smem);
    const int tid = threadIdx.x;
    const int stid = sw(tid);
    // tiles with stride gridDim.x: the co-resident workgroups work on
    // neighbouring tiles at any moment, and neighbouring tiles interleave in
    // memory (at 128-byte granularity when the tile holds qubits 0 and 1), so
    // their loads and stores share DRAM pages
    const int total = grp.first_block[grp.ngroups];
    int blk = blockIdx.x;
    if (blk >= total) return;
    TileLoc cur = locate_tile<T, K, BLOCK>(descs, grp, blk, tid);
    T pre[PER];
    {
        const __amdgpu_buffer_rsrc_t rs = tile_rsrc(reinterpret_cast<T *>(cur.d->coef) + cur.base);
        const uint64_t qubits = cur.d->qubits;
#pragma unroll
        for (int r = 0; r < PER; ++r) pre[r] = BufIO<T>::ld(rs, cur.voff, stream_soff<T, K, BLOCK>(qubits, r));
#pragma unroll
        for (int r = 0; r < PER; ++r) lc[stid ^ sw(r * BLOCK)] = pre[r];
    }
    // Per tile: its op list staged (unless it is already in oc), the next
    // tile's early rows' loads (FP64: and its op list), the ops in LDS,
    // (FP64) the late rows' loads, this tile's stores, then the wait for the
    // loads.  Loads and stores share one
    // counter that completes in issue order, so with every load issued
    // before the stores that wait does not cover the stores.
    const TilePassDesc *cached = nullptr;  // descriptor whose whole op list is in oc
    long long tcount = 0, updates = 0;
    // FP64: the next tile's op list comes into registers (one 16-byte op
    // per lane of wave 0) with its first rows and goes to oc after this
    // tile's last barrier.  A workgroup's consecutive tiles lie gridDim.x
    // apart, in other circuits' passes, so staging at the top of the loop
    // put a global round trip before every tile's ops.  The maps are not
    // copied: the streaming sweeps read them by scalar loads.  FP32 keeps
    // its whole-tile prefetch instead (the op words would not fit beside it).
    constexpr bool kOpPrefetch = sizeof(T) == 8;
    typedef unsigned OpW __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) OpW *GOpW;
    OpW opw = {0u, 0u, 0u, 0u};
    for (;;) {
        const int o0 = cur.d->op_begin, o1 = cur.d->op_end;
        const bool fits = o1 - o0 <= kStreamOps;
        if (cur.d != cached) {
            stage_ops<kStreamOps>(&oc, cur.d->ops, cur.d->maps, o0, fits ? o1 - o0 : kStreamOps, tid, BLOCK);
            cached = fits ? cur.d : nullptr;
        }
        const int nblk = blk + gridDim.x;
        const bool has_next = nblk < total;
        TileLoc nxt = cur;
        // rows of the next tile loaded while the ops run: all of them in
        // FP32; 10 of 16 in FP64, where more beside the op words would push
        // the kernel past 128 VGPRs (three waves per SIMD instead of four,
        // which cost 7 %) or spill; the other rows are loaded as soon as the
        // ops end
        constexpr int PE = sizeof(T) == 8 ? (PER * 10) / 16 : PER;
        bool op_pref = false;  // opw holds the next tile's whole op list
        int next_ops = 0;
        if (has_next) {
            nxt = locate_tile<T, K, BLOCK>(descs, grp, nblk, tid);
            if constexpr (kOpPrefetch) {
                const int n0 = nxt.d->op_begin;
                next_ops = nxt.d->op_end - n0;
                op_pref = nxt.d != cur.d && next_ops <= kStreamOps;
                if (op_pref && tid < next_ops) opw = ((GOpW)nxt.d->ops)[n0 + tid];
                else opw = OpW{0u, 0u, 0u, 0u};
            }
            const __amdgpu_buffer_rsrc_t rs = tile_rsrc(reinterpret_cast<T *>(nxt.d->coef) + nxt.base);
            const uint64_t qubits = nxt.d->qubits;
#pragma unroll
            for (int r = 0; r < PE; ++r) pre[r] = BufIO<T>::ld(rs, nxt.voff, stream_soff<T, K, BLOCK>(qubits, r));
        }
        run_ops<T, false, K, BLOCK, kStreamOps>(lc, nullptr, cur.d->ops, cur.d->maps, o0, o1, tcount, updates, redi, &oc,
                                                true);
        if (!fits) cached = nullptr;  // run_ops reloaded later chunks into oc
        if constexpr (PE < PER) {
            if (has_next) {
                const __amdgpu_buffer_rsrc_t rs = tile_rsrc(reinterpret_cast<T *>(nxt.d->coef) + nxt.base);
                const uint64_t qubits = nxt.d->qubits;
#pragma unroll
                for (int r = PE; r < PER; ++r) pre[r] = BufIO<T>::ld(rs, nxt.voff, stream_soff<T, K, BLOCK>(qubits, r));
            } else {
                // a constant, not the previous rows: keeping those as the
                // merge's other input would hold their registers across the ops
#pragma unroll
                for (int r = PE; r < PER; ++r) pre[r] = T(0);
            }
        }
        T out[PER];
        // an opaque copy of the slot base: the 16 tile addresses are
        // recomputed per tile (16 XORs) instead of living in 16 VGPRs
        // across the whole loop
        int st = stid;
        __asm__ volatile("" : "+v"(st));
#pragma unroll
        for (int r = 0; r < PER; ++r) out[r] = lc[st ^ sw(r * BLOCK)];
        {
            const __amdgpu_buffer_rsrc_t rs = tile_rsrc(reinterpret_cast<T *>(cur.d->coef) + cur.base);
            const uint64_t qubits = cur.d->qubits;
#pragma unroll
            for (int r = 0; r < PER; ++r) BufIO<T>::st(rs, cur.voff, stream_soff<T, K, BLOCK>(qubits, r), out[r]);
        }
        if (!has_next) break;
        lds_barrier();  // every thread has read this tile and is done with oc
        if (op_pref) {
            if (tid < next_ops) reinterpret_cast<OpW *>(oc.ops)[tid] = opw;
            cached = nxt.d;  // published by run_ops' first barrier
        }
        st = stid;
        __asm__ volatile("" : "+v"(st));
#pragma unroll
        for (int r = 0; r < PER; ++r) lc[st ^ sw(r * BLOCK)] = pre[r];
        blk = nblk;
        cur = nxt;
    }
}

// --------------------------------------------------- register tile kernel
// One wave per 4^6-slot tile, the tile held in registers as FP64: lane l and
// register e hold the slot whose local digits are the lane digits
// (l0, l1, l2) = (l & 3, (l >> 2) & 3, l >> 4) and the register digits
// (t0, t1, t2) = (e & 3, (e >> 2) & 3, e >> 4) of the current layout
// (t0 < t1 < t2, l0 < l1 < l2 the other three).  The ops of a SEG segment act
// on its register digits only, so a U1 is 16 register quads times a 3x3 map
// and a CX is a fixed set of register moves; between segments the tile is
// re-laid through LDS.  A layout whose register digits avoid local digits 0
// and 1 has lanes 0-15 on 16 consecutive slots (128 bytes) and is loaded from
// and stored to HBM directly.  Ops run in list order with the same FP64
// expressions as the LDS kernels; FP32 weights are rounded where those
// kernels store to LDS (after every op outside a GROUP and at the end of each
// GROUP), so every launch shape gives bit-identical weights.
struct RegLayout {
    int t0, t1, t2, l0, l1, l2;
};

__device__ __forceinline__ RegLayout reg_layout(unsigned triple) {
    RegLayout L;
    unsigned t = triple;
    L.t0 = __builtin_ctz(t);
    t &= t - 1;
    L.t1 = __builtin_ctz(t);
    t &= t - 1;
    L.t2 = __builtin_ctz(t);
    unsigned r = 0x3fu & ~triple;
    L.l0 = __builtin_ctz(r);
    r &= r - 1;
    L.l1 = __builtin_ctz(r);
    r &= r - 1;
    L.l2 = __builtin_ctz(r);
    return L;
}

// LDS word of the local index whose digit j is d, XOR-combined over digits.
// The low four bits (the 8-byte bank) get a linear function of the digits
// such that, read as GF(4)^2 = {(u, v)}, digits 0..5 contribute along the
// lines {(x, 0)}, {(0, x)}, {(x, x)}, {(x, w x)}, {(x, w^2 x)}, {(x, w^2 x)};
// distinct lines meet only in 0, so the 16 values of any two digits other
// than the pair (4, 5) land on 16 distinct banks.  The first two lane digits
// of a layout are never (4, 5), so every 16-lane quarter of a wave's access
// is conflict-free.  The map is a bijection (bits 4 and up are kept).
__device__ __forceinline__ int rsw_digit(int j, int d) {
    const int w1 = ((d >> 1) & 1) | (((d ^ (d >> 1)) & 1) << 1);  // w d
    const int w2 = ((d ^ (d >> 1)) & 1) | ((d & 1) << 1);         // w^2 d
    const int v = j == 2 ? d : (j == 3 ? w1 : w2);
    return (d << (2 * j)) ^ (j >= 2 ? (d | (v << 2)) : 0);
}

__device__ __forceinline__ int reg_lane_word(const RegLayout &L, int lane) {
    return rsw_digit(L.l0, lane & 3) ^ rsw_digit(L.l1, (lane >> 2) & 3) ^ rsw_digit(L.l2, lane >> 4);
}

// e -> XOR of the basis words of its six bits (uniform)
struct RegBasis {
    int w[6];
};
__device__ __forceinline__ RegBasis reg_basis(const RegLayout &L) {
    return RegBasis{{rsw_digit(L.t0, 1), rsw_digit(L.t0, 2), rsw_digit(L.t1, 1), rsw_digit(L.t1, 2),
                     rsw_digit(L.t2, 1), rsw_digit(L.t2, 2)}};
}
__device__ __forceinline__ int reg_word(const RegBasis &B, int e) {
    int o = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
        if ((e >> j) & 1) o ^= B.w[j];
    return o;
}

template <typename T>
__device__ __forceinline__ void reg_relayout(double (&v)[64], T *lds, const RegLayout &A, const RegLayout &B,
                                             int lane) {
    // byte addresses: (word ^ word) * sizeof(T) = (bytes ^ bytes)
    constexpr int S = sizeof(T) == 8 ? 3 : 2;
    char *base = reinterpret_cast<char *>(lds);
    {
        const int lw = reg_lane_word(A, lane) << S;
        RegBasis rb = reg_basis(A);
#pragma unroll
        for (int j = 0; j < 6; ++j) rb.w[j] <<= S;
#pragma unroll
        for (int e = 0; e < 64; ++e) *reinterpret_cast<T *>(base + (lw ^ reg_word(rb, e))) = (T)v[e];
    }
    lds_barrier();
    {
        const int lw = reg_lane_word(B, lane) << S;
        RegBasis rb = reg_basis(B);
#pragma unroll
        for (int j = 0; j < 6; ++j) rb.w[j] <<= S;
#pragma unroll
        for (int e = 0; e < 64; ++e) v[e] = (double)*reinterpret_cast<const T *>(base + (lw ^ reg_word(rb, e)));
    }
    lds_barrier();
}

// Global slot offsets of a layout (lanes 0-15 must be local digits 0 and 1).
struct RegGlobal {
    long long lane;
    long long w[6];
};
__device__ __forceinline__ RegGlobal reg_global(const RegLayout &L, uint64_t qubits, int lane) {
    auto gq = [&](int j) { return 2 * (int)((qubits >> (8 * j)) & 0xff); };
    RegGlobal G;
    G.lane = ((long long)(lane & 3) << gq(L.l0)) | ((long long)((lane >> 2) & 3) << gq(L.l1)) |
             ((long long)(lane >> 4) << gq(L.l2));
    G.w[0] = 1ll << gq(L.t0);
    G.w[1] = 2ll << gq(L.t0);
    G.w[2] = 1ll << gq(L.t1);
    G.w[3] = 2ll << gq(L.t1);
    G.w[4] = 1ll << gq(L.t2);
    G.w[5] = 2ll << gq(L.t2);
    return G;
}
__device__ __forceinline__ long long reg_goff(const RegGlobal &G, int e) {
    long long o = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
        if ((e >> j) & 1) o += G.w[j];
    return o;
}

// U1 on register digit P: the quads e + {1, 2, 3} * 4^P (X, Z, Y).
template <int P>
__device__ __forceinline__ void reg_u1(double (&v)[64], const double *__restrict__ M) {
    constexpr int S = 1 << (2 * P);
    const double m00 = M[0], m01 = M[1], m02 = M[2];
    const double m10 = M[3], m11 = M[4], m12 = M[5];
    const double m20 = M[6], m21 = M[7], m22 = M[8];
#pragma unroll
    for (int e = 0; e < 64; ++e) {
        if ((e >> (2 * P)) & 3) continue;
        const double cx = v[e + S], cz = v[e + 2 * S], cy = v[e + 3 * S];
        v[e + S] = map_row(m00, m01, m02, cx, cy, cz);
        v[e + 3 * S] = map_row(m10, m11, m12, cx, cy, cz);
        v[e + 2 * S] = map_row(m20, m21, m22, cx, cy, cz);
    }
}

template <int PC, int PT, int P>
__device__ __forceinline__ void reg_cx_pair(double (&v)[64]) {
    constexpr CxPairC pr = cx_pair_c(P);
    constexpr int PR = 3 - PC - PT;
#pragma unroll
    for (int dr = 0; dr < 4; ++dr) {
        const int e1 = (pr.dc1 << (2 * PC)) | (pr.dt1 << (2 * PT)) | (dr << (2 * PR));
        const int e2 = (pr.dc2 << (2 * PC)) | (pr.dt2 << (2 * PT)) | (dr << (2 * PR));
        const double t1 = v[e1], t2 = v[e2];
        v[e1] = pr.neg ? -t2 : t2;
        v[e2] = pr.neg ? -t1 : t1;
    }
}

// CX with control on register digit PC and target on PT.
template <int PC, int PT>
__device__ __forceinline__ void reg_cx(double (&v)[64]) {
    reg_cx_pair<PC, PT, 0>(v);
    reg_cx_pair<PC, PT, 1>(v);
    reg_cx_pair<PC, PT, 2>(v);
    reg_cx_pair<PC, PT, 3>(v);
    reg_cx_pair<PC, PT, 4>(v);
    reg_cx_pair<PC, PT, 5>(v);
}

__device__ __forceinline__ double lane_read_f64(double x, int lane) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ void reg_round(double (&v)[64]) {
    if constexpr (!std::is_same<T, double>::value) {
#pragma unroll
        for (int e = 0; e < 64; ++e) v[e] = (double)(T)v[e];
    }
}

// Where a tile of a launch lives: its descriptor fields and slot base.
struct RegTile {
    void *coef;
    const DOp *ops;
    const double *maps;
    long long base;
    uint64_t qubits;
    int o0, o1;
    unsigned entry;
};

__device__ __forceinline__ RegTile reg_locate(const TilePassDesc *__restrict__ descs, const TileGroups &grp, int b) {
    int gi = 0;
    while (gi + 1 < grp.ngroups && b >= grp.first_block[gi + 1]) ++gi;
    const int rel = b - grp.first_block[gi];
    const TilePassDesc &d = descs[grp.first_desc[gi] + (rel >> grp.shift[gi])];
    RegTile t;
    t.coef = d.coef;
    t.ops = d.ops;
    t.maps = d.maps;
    t.qubits = d.qubits;
    t.o0 = d.op_begin;
    t.o1 = d.op_end;
    t.entry = d.reg_entry;
    if (__builtin_popcount(t.entry) != 3 || (t.entry & ~0x3cu)) t.entry = 0x38u;
    unsigned inmask = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) inmask |= 1u << (unsigned)((t.qubits >> (8 * j)) & 0xff);
    long long base = 0, rest = rel & ((1 << grp.shift[gi]) - 1);
    const int n = d.n;
    for (int q = 0; q < n; ++q) {
        if ((inmask >> q) & 1u) continue;
        base |= (rest & 3ll) << (2 * q);
        rest >>= 2;
    }
    t.base = base;
    return t;
}

// Op entries [cb, cb + 64) of a pass, one per lane, with the map of a U1.
struct RegOps {
    uint32_t w0, w1, w2;
    double m[9];
};
__device__ __forceinline__ void reg_load_ops(RegOps &r, const RegTile &t, int cb, int lane) {
    const int i = cb + lane;
    if (i < t.o1) {
        const uint32_t *w = reinterpret_cast<const uint32_t *>(t.ops + i);
        r.w0 = w[0];
        r.w1 = w[1];
        r.w2 = w[2];
        if ((r.w0 & 0xff) == DOP_U1) {
            const double *src = t.maps + 9ull * r.w2;
#pragma unroll
            for (int j = 0; j < 9; ++j) r.m[j] = src[j];
        }
    }
}

template <typename T, typename V>
__device__ __forceinline__ void reg_load_tile(V (&v)[64], const RegTile &t, int lane) {
    const RegLayout L = reg_layout(t.entry);
    const RegGlobal G = reg_global(L, t.qubits, lane);
    const __amdgpu_buffer_rsrc_t rs = tile_rsrc(reinterpret_cast<T *>(t.coef) + t.base);
    const unsigned lo = (unsigned)G.lane * (unsigned)sizeof(T);
#pragma unroll
    for (int e = 0; e < 64; ++e) v[e] = (V)BufIO<T>::ld(rs, lo, (unsigned)reg_goff(G, e) * (unsigned)sizeof(T));
}

// Persistent: a grid of at most (co-resident waves) single-wave workgroups
// walks the launch's tiles with stride gridDim.x; while a wave runs the ops
// of one tile, the loads of its next tile (and that pass's op entries) are
// in flight, so HBM latency overlaps the register work.
template <typename T, bool PF>
__global__ __launch_bounds__(64) void tile_reg_kernel(const TilePassDesc *__restrict__ descs, TileGroups grp) {
    __shared__ __align__(16) T lds[1 << 12];  // the launch's only LDS: byte address = offset
    const int total = grp.first_block[grp.ngroups];
    const int lane = threadIdx.x;
    int blk = blockIdx.x;
    if (blk >= total) return;
    RegTile cur = reg_locate(descs, grp, blk);
    RegOps oc;
    oc.w0 = oc.w1 = oc.w2 = 0;
#pragma unroll
    for (int j = 0; j < 9; ++j) oc.m[j] = 0.0;
    reg_load_ops(oc, cur, cur.o0, lane);
    double v[64];
    reg_load_tile<T>(v, cur, lane);
    for (;;) {
        const int nblk = blk + (int)gridDim.x;
        const bool has_next = nblk < total;
        RegTile nxt = cur;
        RegOps on = oc;
        T pre[64];
        if (has_next) {
            nxt = reg_locate(descs, grp, nblk);
            if (PF) {
                reg_load_ops(on, nxt, nxt.o0, lane);
                reg_load_tile<T>(pre, nxt, lane);
            }
        }
        // ---- the ops of the current tile, in registers: one flat dispatch
        // per entry (a single join point keeps one register assignment)
        constexpr unsigned kHbmTriple = 0x38u;  // digits 3, 4, 5 in registers
        unsigned lay = cur.entry;
        RegLayout L = reg_layout(lay);
        int cb = cur.o0, grp_left = 0;
        for (int i = cur.o0; i < cur.o1; ++i) {
            if (i - cb >= 64) {
                cb = i;
                reg_load_ops(oc, cur, cb, lane);
            }
            const int li = i - cb;
            const uint32_t w0 = __builtin_amdgcn_readlane(oc.w0, li);
            const int kind = w0 & 0xff, a = (w0 >> 8) & 0xff, bd = (w0 >> 16) & 0xff;
            int code = 0;  // 0 nothing, 1-3 U1 on register digit 0-2, 4-9 CX, 10 re-layout
            bool rnd = false;
            unsigned next = lay;
            if (kind == DOP_SEG) {
                const uint32_t w1 = __builtin_amdgcn_readlane(oc.w1, li);
                next = (1u << a) | (1u << bd) | (1u << (w1 & 0xffff));
                code = next != lay ? 10 : 0;
            } else if (kind == DOP_GROUP) {
                grp_left = (w0 >> 24) & 0xff;
            } else {
                const int pa = a == L.t0 ? 0 : (a == L.t1 ? 1 : 2);
                if (kind == DOP_U1) {
                    code = 1 + pa;
                } else {
                    const int pb = bd == L.t0 ? 0 : (bd == L.t1 ? 1 : 2);
                    // (pa, pb) = (0,1) (0,2) (1,0) (1,2) (2,0) (2,1) -> 4..9
                    code = 4 + 2 * pa + (pb > pa ? pb - 1 : pb);
                }
                if (grp_left > 0) rnd = --grp_left == 0;
                else rnd = kind == DOP_U1;
            }
            double M[9];
            if (code >= 1 && code <= 3) {
#pragma unroll
                for (int j = 0; j < 9; ++j) M[j] = lane_read_f64(oc.m[j], li);
            }
            switch (code) {
            case 1: reg_u1<0>(v, M); break;
            case 2: reg_u1<1>(v, M); break;
            case 3: reg_u1<2>(v, M); break;
            case 4: reg_cx<0, 1>(v); break;
            case 5: reg_cx<0, 2>(v); break;
            case 6: reg_cx<1, 0>(v); break;
            case 7: reg_cx<1, 2>(v); break;
            case 8: reg_cx<2, 0>(v); break;
            case 9: reg_cx<2, 1>(v); break;
            case 10: {
                const RegLayout N = reg_layout(next);
                reg_relayout<T>(v, lds, L, N, lane);
                L = N;
                lay = next;
                break;
            }
            default: break;
            }
            if (rnd) reg_round<T>(v);
        }
        if (lay & 3u) {
            const RegLayout N = reg_layout(kHbmTriple);
            reg_relayout<T>(v, lds, L, N, lane);
            L = N;
        }
        {
            const RegGlobal G = reg_global(L, cur.qubits, lane);
            const __amdgpu_buffer_rsrc_t rs = tile_rsrc(reinterpret_cast<T *>(cur.coef) + cur.base);
            const unsigned lo = (unsigned)G.lane * (unsigned)sizeof(T);
#pragma unroll
            for (int e = 0; e < 64; ++e) BufIO<T>::st(rs, lo, (unsigned)reg_goff(G, e) * (unsigned)sizeof(T), (T)v[e]);
        }
        if (!has_next) break;
        blk = nblk;
        cur = nxt;
        if (PF) {
            oc = on;
#pragma unroll
            for (int e = 0; e < 64; ++e) v[e] = (double)pre[e];
        } else {
            reg_load_ops(oc, cur, cur.o0, lane);
            reg_load_tile<T>(v, cur, lane);
        }
    }
}

// ------------------------------------------------------ adjoint sweep
// Forward propagation of the observable weights c and the state
// coefficients r through one pass.  U1 ops hold the Heisenberg matrix M of a
// single gate; the forward map (Table I) is its transpose because the maps
// are orthogonal.  For a rotation R_sigma(theta) the derivative of <O> is
// c^T (0 + A_sigma) r taken just before the gate, where A_sigma = R'(0) is the
// generator of the forward rotation on (X, Y, Z):
//   RX: c_Z r_Y - c_Y r_Z,  RY: c_X r_Z - c_Z r_X,  RZ: c_Y r_X - c_X r_Y.
template <int K, int BLOCK>
__device__ double join_part(const double *lc, const double *lr, int a, int axis, int tid) {
    constexpr int NQ = 1 << (2 * (K - 1));
    const int sh = 2 * a;
    const int lowmask = (1 << sh) - 1;
    double acc = 0.0;
    for (int u = tid; u < NQ; u += BLOCK) {
        const int base = ((u & ~lowmask) << 2) | (u & lowmask);
        const int iX = sw(base | (1 << sh)), iZ = sw(base | (2 << sh)), iY = sw(base | (3 << sh));
        if (axis == 3) acc += lc[iZ] * lr[iY] - lc[iY] * lr[iZ];
        else if (axis == 4) acc += lc[iX] * lr[iZ] - lc[iZ] * lr[iX];
        else acc += lc[iY] * lr[iX] - lc[iX] * lr[iY];
    }
    return acc;
}

template <int K, int BLOCK>
__global__ __launch_bounds__(BLOCK) void grad_kernel(const GradPassDesc *__restrict__ desc) {
    extern __shared__ __align__(256) unsigned char smem[];
    __shared__ double redd[BLOCK / 64];
    __shared__ OpCache oc;
    const GradPassDesc d = *desc;
    constexpr int size = 1 << (2 * K);
    double *lc = reinterpret_cast<double *>(smem);
    double *lr = lc + size;
    const int tid = threadIdx.x;
    const long long tile = blockIdx.x;
    unsigned inmask = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < K) inmask |= 1u << (unsigned)((d.qubits >> (8 * j)) & 0xff);
    long long base = 0;
    {
        long long t = tile;
        for (int q = 0; q < d.n; ++q) {
            if ((inmask >> q) & 1u) continue;
            base |= (t & 3ll) << (2 * q);
            t >>= 2;
        }
    }
    for (int i = tid; i < size; i += BLOCK) {
        const long long gi = base | deposit_digits(i, d.qubits, 0, K);
        lc[sw(i)] = d.c[gi];
        lr[sw(i)] = d.r[gi];
    }
    for (int cb = d.op_begin; cb < d.op_end; cb += OPCH) {
        const int cn = (d.op_end - cb) < OPCH ? (d.op_end - cb) : OPCH;
        lds_barrier();
        stage_ops<OPCH>(&oc, d.ops, d.maps, cb, cn, tid, BLOCK);
        lds_barrier();
        for (int i = 0; i < cn; ++i) {
            const uint32_t w0 = __builtin_amdgcn_readfirstlane(reinterpret_cast<const uint32_t *>(&oc.ops[i])[0]);
            const uint32_t slot = __builtin_amdgcn_readfirstlane(reinterpret_cast<const uint32_t *>(&oc.ops[i])[3]);
            const int kind = w0 & 0xff, a = (w0 >> 8) & 0xff, b = (w0 >> 16) & 0xff;
            if (kind == DOP_U1) {
                if (b >= 3) {
                    const double part = block_sum_d<BLOCK>(join_part<K, BLOCK>(lc, lr, a, b, tid), redd);
                    if (tid == 0) d.partials[(long long)(slot - d.slot_base) * d.ntiles + tile] = part;
                    lds_barrier();
                }
                const double *M = oc.maps[i];
                const double Mt[9] = {M[0], M[3], M[6], M[1], M[4], M[7], M[2], M[5], M[8]};
                u1_apply<double, false, K, BLOCK>(lc, nullptr, a, Mt, 0u, tid);
                u1_apply<double, false, K, BLOCK>(lr, nullptr, a, Mt, 0u, tid);
            } else {
                if constexpr (K >= 2) {
                    cx_apply<double, false, K, BLOCK>(lc, nullptr, a, b, tid);
                    cx_apply<double, false, K, BLOCK>(lr, nullptr, a, b, tid);
                }
            }
            lds_barrier();
        }
    }
    lds_barrier();
    for (int i = tid; i < size; i += BLOCK) {
        const long long gi = base | deposit_digits(i, d.qubits, 0, K);
        d.c[gi] = lc[sw(i)];
        d.r[gi] = lr[sw(i)];
    }
}

// r of |0...0><0...0|: Tr(P rho) = 1 for strings of I and Z only, else 0
__global__ void grad_init_state_kernel(double *r, int n, long long size) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < size;
         i += (long long)gridDim.x * blockDim.x) {
        bool zonly = true;
        for (int q = 0; q < n; ++q) zonly = zonly && !((i >> (2 * q)) & 1);
        r[i] = zonly ? 1.0 : 0.0;
    }
}

__global__ void grad_reduce_kernel(const double *partials, int nslots, int ntiles, double *rot_grad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nslots) return;
    double s = 0.0;
    for (int t = 0; t < ntiles; ++t) s += partials[(long long)j * ntiles + t];
    rot_grad[j] = s;
}

// sequential so that gates sharing a parameter are summed in gate order
__global__ void grad_accumulate_kernel(const double *rot_grad, const int32_t *slot_param, int nslots, double *grad,
                                       int nparams) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int p = 0; p < nparams; ++p) grad[p] = 0.0;
    for (int j = 0; j < nslots; ++j) grad[slot_param[j]] += rot_grad[j];
}

__global__ void copy_f64_n_kernel(const double *src, double *dst, long long count) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ------------------------------------------------------- density matrix
// rho = 2^-n sum_Q r_Q Q from the Pauli weights r of 2^n rho (slot order; the
// sum form of the density operator over the stabilizer group, eq. (3)).  A
// string Q = (x, z) with Y = iXZ has one nonzero per column (Sec. III-D):
// <a|Q|b> = [a = b ^ x] i^|x & z| (-1)^|b & z|.  So for a fixed x the column
// entries rho[b ^ x][b] over all b are the Walsh-Hadamard transform over z of
// r(x, z) i^|x & z|.  Workgroup x gathers those 2^n weights into LDS (real
// and imaginary parts), runs the n butterfly stages and writes its 2^n
// entries.  rho is row-major complex (re, im) doubles, rho[a][b] at
// 2 (a 2^n + b); basis bit q is qubit q.
__device__ __forceinline__ unsigned long long spread_bits(unsigned v) {
    unsigned long long r = 0;
    for (int q = 0; v; ++q, v >>= 1) r |= (unsigned long long)(v & 1u) << (2 * q);
    return r;
}

template <typename T>
__global__ __launch_bounds__(256) void density_decode_kernel(const T *__restrict__ coef, int n,
                                                             double *__restrict__ rho) {
    extern __shared__ __align__(256) unsigned char smem[];
    const int N = 1 << n;
    double *re = reinterpret_cast<double *>(smem);
    double *im = re + N;
    const unsigned x = blockIdx.x;
    const unsigned long long sx = spread_bits(x);
    for (int z = threadIdx.x; z < N; z += blockDim.x) {
        const double w = (double)coef[sx | (spread_bits((unsigned)z) << 1)];
        const int k = __popc(x & (unsigned)z) & 3;  // the phase i^k
        re[z] = k == 0 ? w : (k == 2 ? -w : 0.0);
        im[z] = k == 1 ? w : (k == 3 ? -w : 0.0);
    }
    __syncthreads();
    for (int h = 1; h < N; h <<= 1) {
        for (int t = threadIdx.x; t < N / 2; t += blockDim.x) {
            const int i = ((t & ~(h - 1)) << 1) | (t & (h - 1)), j = i | h;
            const double a = re[i], b = re[j], c = im[i], d = im[j];
            re[i] = a + b;
            re[j] = a - b;
            im[i] = c + d;
            im[j] = c - d;
        }
        __syncthreads();
    }
    const double scale = 1.0 / (double)N;
    for (int b = threadIdx.x; b < N; b += blockDim.x) {
        const size_t e = 2 * ((size_t)((unsigned)b ^ x) * (size_t)N + (size_t)b);
        rho[e] = re[b] * scale;
        rho[e + 1] = im[b] * scale;
    }
}

hipError_t launch_density_decode(const void *coef, int n, int dtype_bytes, double *rho, hipStream_t s) {
    if (n < 1 || n > 12) return hipErrorInvalidValue;
    const size_t lds = (size_t)2 * ((size_t)1 << n) * sizeof(double);
    const dim3 grid(1u << n), block(n >= 8 ? 256 : 64);
    if (dtype_bytes == 8) {
        static bool attr = false;
        if (!attr) {
            hipError_t e = hipFuncSetAttribute((const void *)density_decode_kernel<double>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
            if (e != hipSuccess) return e;
            attr = true;
        }
        hipLaunchKernelGGL(density_decode_kernel<double>, grid, block, lds, s, (const double *)coef, n, rho);
    } else {
        static bool attr = false;
        if (!attr) {
            hipError_t e = hipFuncSetAttribute((const void *)density_decode_kernel<float>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
            if (e != hipSuccess) return e;
            attr = true;
        }
        hipLaunchKernelGGL(density_decode_kernel<float>, grid, block, lds, s, (const float *)coef, n, rho);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------- map composer
// maps[i] = G_last * ... * G_first over the recipe of op i, where G is the
// Heisenberg matrix of one gate acting on the (X, Y, Z) weights:
//   RX: Y -> cY - sZ, Z -> cZ + sY     RY: X -> cX + sZ, Z -> cZ - sX
//   RZ: X -> cX - sY, Y -> cY + sX     H: X <-> Z, Y -> -Y
//   S:  X -> -Y, Y -> X   (S^dag P S; the forward Table I row inverted)
__device__ void gate_matrix(int op, double th, double G[9]) {
    for (int i = 0; i < 9; ++i) G[i] = 0.0;
    double s = 0.0, c = 1.0;
    if (op >= 3) sincos(th, &s, &c);
    switch (op) {
    case 0: G[2] = 1; G[4] = -1; G[6] = 1; break;               // H
    case 1: G[1] = 1; G[3] = -1; G[8] = 1; break;               // S
    case 3: G[0] = 1; G[4] = c; G[5] = s; G[7] = -s; G[8] = c; break;  // RX
    case 4: G[0] = c; G[2] = -s; G[4] = 1; G[6] = s; G[8] = c; break;  // RY
    default: G[0] = c; G[1] = s; G[3] = -s; G[4] = c; G[8] = 1; break; // RZ
    }
}

// Maps are composed by one lane when their recipe is short and by a whole
// wave when it is long (the rule depends on the map alone, so a circuit's
// maps are the same bits however it is batched).  A wave takes 64
// consecutive maps: each lane folds its short recipe in order; then for each
// long recipe of the 64, the lanes build the matrices of 64 consecutive
// gates at once (their parameter loads and sincos in parallel), an ordered
// tree of 3x3 products over the lanes multiplies them (later gates on the
// left), and the chunk products are applied in recipe order.  Block (d, y)
// serves descriptor d; its y blocks and their waves share its maps.
constexpr int kShortRecipe = 8;

__device__ __forceinline__ void mat3_mul(const double A[9], const double B[9], double C[9]) {
    // C = A * B
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) C[3 * a + b] = A[3 * a] * B[b] + A[3 * a + 1] * B[3 + b] + A[3 * a + 2] * B[6 + b];
}

// A descriptor with reserved = 1 composes forward maps (P -> g P g^dag): the
// transpose of each gate's Heisenberg matrix, since the maps are orthogonal.
__device__ __forceinline__ void gate_matrix_dir(int op, double th, bool fwd, double G[9]) {
    gate_matrix(op, th, G);
    if (fwd) {
        double t;
        t = G[1]; G[1] = G[3]; G[3] = t;
        t = G[2]; G[2] = G[6]; G[6] = t;
        t = G[5]; G[5] = G[7]; G[7] = t;
    }
}

__global__ __launch_bounds__(256) void compose_kernel(const ComposeDesc *__restrict__ descs) {
    const ComposeDesc &d = descs[blockIdx.x];
    const bool fwd = d.reserved == 1;
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int wstride = gridDim.y * wpb;
    for (int w0 = (blockIdx.y * wpb + (threadIdx.x >> 6)) * 64; w0 < d.nmaps; w0 += wstride * 64) {
        const int i = w0 + lane;
        bool longr = false;
        if (i < d.nmaps) {
            const int r0 = d.roff[i], r1 = d.roff[i + 1];
            longr = r1 - r0 > kShortRecipe;
            if (!longr) {
                double M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
                for (int r = r0; r < r1; ++r) {
                    const int op = d.rop[r];
                    double G[9], P[9];
                    gate_matrix_dir(op, op >= 3 ? d.theta[d.rparam[r]] : 0.0, fwd, G);
                    mat3_mul(G, M, P);
                    for (int t = 0; t < 9; ++t) M[t] = P[t];
                }
                for (int t = 0; t < 9; ++t) d.maps[9ull * i + t] = M[t];
            }
        }
        uint64_t todo = __ballot(longr);
        while (todo) {
            const int l = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int m = w0 + l;
            const int r0 = d.roff[m], r1 = d.roff[m + 1];
            double M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
            for (int c0 = r0; c0 < r1; c0 += 64) {
                double G[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
                const int r = c0 + lane;
                if (r < r1) {
                    const int op = d.rop[r];
                    gate_matrix_dir(op, op >= 3 ? d.theta[d.rparam[r]] : 0.0, fwd, G);
                }
                // lane l holds the product of gates [c0 + l, c0 + l + w) after
                // the step of width w; combine with the next block on the left
#pragma unroll
                for (int w = 1; w < 64; w <<= 1) {
                    double B[9], C[9];
#pragma unroll
                    for (int t = 0; t < 9; ++t) B[t] = __shfl_down(G[t], w, 64);
                    mat3_mul(B, G, C);
                    if ((lane & (2 * w - 1)) == 0) {
#pragma unroll
                        for (int t = 0; t < 9; ++t) G[t] = C[t];
                    }
                }
                double P[9], C[9];
#pragma unroll
                for (int t = 0; t < 9; ++t) P[t] = __shfl(G[t], 0, 64);
                mat3_mul(P, M, C);
#pragma unroll
                for (int t = 0; t < 9; ++t) M[t] = C[t];
            }
            if (lane == 0) {
#pragma unroll
                for (int t = 0; t < 9; ++t) d.maps[9ull * m + t] = M[t];
            }
        }
    }
}

// -------------------------------------------------------- small kernels
template <typename T>
__global__ void dense_fill_kernel(T *coef, uint8_t *pres, long long size) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < size;
         i += (long long)gridDim.x * blockDim.x) {
        coef[i] = (T)0;
        if (pres) pres[i] = 0;
    }
}

// Sequential so that repeated strings are summed in input order; block b
// fills the weights at coef + b * stride (one block per parameter set).
template <typename T>
__global__ void dense_scatter_kernel(T *coef, uint8_t *pres, int n, const uint64_t *x, const uint64_t *z,
                                     const double *c, int nterms, long long stride) {
    if (threadIdx.x != 0) return;
    coef += blockIdx.x * stride;
    for (int t = 0; t < nterms; ++t) {
        const long long s = morton_slot(x[t], z[t], n);
        coef[s] = (T)((double)coef[s] + c[t]);
        if (pres) pres[s] = 1;
    }
}

// Block b reads out the weights at coef + b * stride into out[b]; the same
// fixed-order reduction for one evaluation or many.
template <typename T>
__global__ __launch_bounds__(256) void dense_readout_kernel(const T *coef, int n, double *out, long long stride) {
    __shared__ double redd[4];
    coef += blockIdx.x * stride;
    double part = 0.0;
    for (long long j = threadIdx.x; j < (1ll << n); j += 256) part += (double)coef[zonly_slot(j, n)];
    const double tot = block_sum_d<256>(part, redd);
    if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

template <typename T>
__global__ void many_fill_kernel(const DenseIODesc *__restrict__ descs) {
    const DenseIODesc &d = descs[blockIdx.y];
    T *coef = reinterpret_cast<T *>(d.coef);
    const long long size = 1ll << (2 * d.n);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < size;
         i += (long long)gridDim.x * blockDim.x)
        coef[i] = (T)0;
}

template <typename T>
__global__ void many_scatter_kernel(const DenseIODesc *__restrict__ descs) {
    if (threadIdx.x != 0) return;
    const DenseIODesc &d = descs[blockIdx.x];
    T *coef = reinterpret_cast<T *>(d.coef);
    for (int t = 0; t < d.nterms; ++t) {
        const long long s = morton_slot(d.obs_x[t], d.obs_z[t], d.n);
        coef[s] = (T)((double)coef[s] + d.obs_c[t]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void many_readout_kernel(const DenseIODesc *__restrict__ descs) {
    __shared__ double redd[4];
    const DenseIODesc &d = descs[blockIdx.x];
    const T *coef = reinterpret_cast<const T *>(d.coef);
    double part = 0.0;
    for (long long j = threadIdx.x; j < (1ll << d.n); j += 256) part += (double)coef[zonly_slot(j, d.n)];
    const double tot = block_sum_d<256>(part, redd);
    if (threadIdx.x == 0) *d.out = tot;
}

__global__ __launch_bounds__(256) void dense_count_kernel(const uint8_t *pres, long long size,
                                                           unsigned long long *out) {
    __shared__ long long redi[4];
    long long mine = 0;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < size; i += (long long)gridDim.x * 256) mine += pres[i];
    const long long tot = block_sum_i<256>(mine, redi);
    if (threadIdx.x == 0 && tot) atomicAdd(out, (unsigned long long)tot);
}

// Ordered compaction of present slots into (x, z, c), three phases:
// per-block counts, one exclusive scan, then ordered writes.
constexpr int CMP_CHUNK = 4096;

// A slot is kept when its presence byte is set, or, without presence bytes
// (untracked runs), when its weight is nonzero.
template <typename T>
__device__ __forceinline__ bool slot_kept(const T *coef, const uint8_t *pres, long long i) {
    return pres ? pres[i] != 0 : coef[i] != (T)0;
}

template <typename T>
__global__ __launch_bounds__(256) void compact_count_kernel(const T *coef, const uint8_t *pres, long long size,
                                                            int *counts) {
    __shared__ long long redi[4];
    const long long b0 = (long long)blockIdx.x * CMP_CHUNK;
    long long mine = 0;
    for (int i = threadIdx.x; i < CMP_CHUNK; i += 256)
        if (b0 + i < size) mine += slot_kept(coef, pres, b0 + i);
    const long long tot = block_sum_i<256>(mine, redi);
    if (threadIdx.x == 0) counts[blockIdx.x] = (int)tot;
}

__global__ void compact_scan_kernel(int *counts, int nblocks, unsigned long long *total) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    long long run = 0;
    for (int b = 0; b < nblocks; ++b) {
        const int c = counts[b];
        counts[b] = (int)run;
        run += c;
    }
    *total = (unsigned long long)run;
}

template <typename T>
__global__ __launch_bounds__(256) void compact_write_kernel(const T *coef, const uint8_t *pres, long long size, int n,
                                                            const int *offsets, uint64_t *xo, uint64_t *zo,
                                                            double *co) {
    __shared__ int wcount[4];
    __shared__ int running;
    const long long b0 = (long long)blockIdx.x * CMP_CHUNK;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) running = offsets[blockIdx.x];
    lds_barrier();
    for (int r = 0; r < CMP_CHUNK; r += 256) {
        const long long i = b0 + r + threadIdx.x;
        const bool p = i < size && slot_kept(coef, pres, i);
        const unsigned long long bal = __ballot(p);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[w] = __popcll(bal);
        lds_barrier();
        int off = running;
        for (int v = 0; v < w; ++v) off += wcount[v];
        if (p) {
            const long long pos = off + below;
            uint64_t x = 0, z = 0;
            for (int q = 0; q < n; ++q) {
                x |= (uint64_t)((i >> (2 * q)) & 1) << q;
                z |= (uint64_t)((i >> (2 * q + 1)) & 1) << q;
            }
            xo[pos] = x;
            zo[pos] = z;
            co[pos] = (double)coef[i];
        }
        lds_barrier();
        if (threadIdx.x == 0) running += wcount[0] + wcount[1] + wcount[2] + wcount[3];
        lds_barrier();
    }
}

// ------------------------------------------------------------ launchers
int max_lds_bytes() {
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    cached = v;
    return v;
}

size_t resident_lds_bytes(int n, int dtype_bytes, bool track) {
    const size_t size = (size_t)1 << (2 * n);
    return size * (size_t)dtype_bytes + (track ? size : 0);
}

hipError_t launch_compose(const ComposeDesc *d_descs, int ndescs, hipStream_t s, int max_maps) {
    if (ndescs <= 0) return hipSuccess;
    // 256 maps per block (64 per wave); enough blocks per descriptor for its
    // maps, at most 1024 across the launch's y dimension
    int ychunks = (max_maps + 255) / 256;
    ychunks = ychunks < 1 ? 1 : (ychunks > 1024 ? 1024 : ychunks);
    if ((long long)ychunks * ndescs > 65536) ychunks = (int)std::max<long long>(1, 65536 / ndescs);
    hipLaunchKernelGGL(compose_kernel, dim3(ndescs, ychunks), dim3(256), 0, s, d_descs);
    return hipGetLastError();
}

template <typename T, bool TRACK, int N, int BLOCK>
static hipError_t launch_res_t(const ResidentDesc *d, int nd, size_t lds, hipStream_t s) {
    auto fn = resident_kernel<T, TRACK, N, BLOCK>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           max_lds_bytes() - (int)kStaticLdsReserve);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(fn, dim3(nd), dim3(BLOCK), lds, s, d);
    return hipGetLastError();
}

static int g_res_block[8] = {64, 64, 64, 64, 64, 512, 512, 1024};
void set_resident_block(int n, int block) {
    if (n >= 5 && n <= 7) g_res_block[n] = block;
}
int resident_block(int n) { return (n >= 1 && n <= 7) ? g_res_block[n] : 64; }

template <typename T, bool TRACK>
static hipError_t launch_res_b(const ResidentDesc *d, int nd, int n, size_t lds, hipStream_t s) {
    const int blk = TRACK ? (n <= 4 ? 64 : n <= 6 ? 256 : 512) : g_res_block[n];
    switch (n) {
    case 1: return launch_res_t<T, TRACK, 1, 64>(d, nd, lds, s);
    case 2: return launch_res_t<T, TRACK, 2, 64>(d, nd, lds, s);
    case 3: return launch_res_t<T, TRACK, 3, 64>(d, nd, lds, s);
    case 4: return launch_res_t<T, TRACK, 4, 64>(d, nd, lds, s);
    case 5:
        if (!TRACK && blk == 512) return launch_res_t<T, TRACK, 5, 512>(d, nd, lds, s);
        if (!TRACK && blk == 1024) return launch_res_t<T, TRACK, 5, 1024>(d, nd, lds, s);
        return launch_res_t<T, TRACK, 5, 256>(d, nd, lds, s);
    case 6:
        if (!TRACK && blk == 512) return launch_res_t<T, TRACK, 6, 512>(d, nd, lds, s);
        if (!TRACK && blk == 1024) return launch_res_t<T, TRACK, 6, 1024>(d, nd, lds, s);
        return launch_res_t<T, TRACK, 6, 256>(d, nd, lds, s);
    default:
        if (!TRACK && blk == 256) return launch_res_t<T, TRACK, 7, 256>(d, nd, lds, s);
        if (!TRACK && blk == 1024) return launch_res_t<T, TRACK, 7, 1024>(d, nd, lds, s);
        return launch_res_t<T, TRACK, 7, 512>(d, nd, lds, s);
    }
}

hipError_t launch_resident(const ResidentDesc *d_descs, int ndescs, int n, int dtype_bytes, bool track,
                           hipStream_t s) {
    if (ndescs <= 0) return hipSuccess;
    if (n < 1 || n > 7) return hipErrorInvalidValue;
    const size_t lds = resident_lds_bytes(n, dtype_bytes, track);
    if (dtype_bytes == 8)
        return track ? launch_res_b<double, true>(d_descs, ndescs, n, lds, s)
                     : launch_res_b<double, false>(d_descs, ndescs, n, lds, s);
    return track ? launch_res_b<float, true>(d_descs, ndescs, n, lds, s)
                 : launch_res_b<float, false>(d_descs, ndescs, n, lds, s);
}

// defaults measured on MI355X: one wave per 4^5-slot tile; persistent
// prefetching workgroups for 4^6- and 4^7-slot tiles
static int g_tile_variant[8] = {0, 0, 0, 0, 0, 2, 1, 1};
void set_tile_kernel_variant(int k, int variant) {
    if (k >= 0 && k < 8) g_tile_variant[k] = variant;
}
int tile_kernel_variant(int k) { return (k >= 0 && k < 8) ? g_tile_variant[k] : 0; }

int num_cus() {
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
        cached = v;
    return cached > 0 ? cached : 256;
}

template <typename T, bool TRACK, int K>
static hipError_t launch_tile_t(const TilePassDesc *d, const TileGroups &grp, size_t lds, hipStream_t s) {
    const int nblocks = grp.first_block[grp.ngroups];
    // the register-tile kernel's 32-bit buffer offsets hold registers of at
    // most 14 qubits; every group of a launch shares one n = k + shift / 2
    int max_n = K;
    for (int gi = 0; gi < grp.ngroups; ++gi) max_n = std::max(max_n, K + grp.shift[gi] / 2);
    if (!TRACK && K == 6 && g_tile_variant[6] == 3 && max_n <= 14) {
        // one wave per tile, tile in registers; LDS only for re-layouts
        hipLaunchKernelGGL((tile_reg_kernel<T, false>), dim3(nblocks), dim3(64), 0, s, d, grp);
        return hipGetLastError();
    }
    if (!TRACK && K == 6 && g_tile_variant[6] == 4 && max_n <= 14) {
        // the same, persistent: as many single-wave workgroups as fit at
        // once, each loading its next tile while it works on the current one
        auto fn = tile_reg_kernel<T, true>;
        static int resident = 0;
        if (!resident) {
            int per_cu = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, 64, 0);
            if (e != hipSuccess) return e;
            resident = std::max(per_cu, 1) * num_cus();
        }
        hipLaunchKernelGGL(fn, dim3(std::min(nblocks, resident)), dim3(64), 0, s, d, grp);
        return hipGetLastError();
    }
    if (!TRACK && K <= 6 && g_tile_variant[K] == 2) {
        auto fn = tile_kernel<T, false, (K <= 6 ? K : 6), 64>;
        static bool attr64 = false;
        if (!attr64) {
            hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               max_lds_bytes() - (int)kStaticLdsReserve);
            if (e != hipSuccess) return e;
            attr64 = true;
        }
        hipLaunchKernelGGL(fn, dim3(nblocks), dim3(64), lds, s, d, grp);
        return hipGetLastError();
    }
    if (!TRACK && g_tile_variant[K] == 1 && max_n <= 14) {
        auto fn = tile_stream_kernel<T, K>;
        constexpr int SB = kStreamBlock<K>;
        static int rb = 0;
        if (!rb) {
            hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               max_lds_bytes() - (int)kStaticLdsReserve);
            if (e != hipSuccess) return e;
            int per_cu = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, SB, lds);
            if (e != hipSuccess) return e;
            rb = std::max(per_cu, 1) * num_cus();
        }
        const int grid = nblocks < rb ? nblocks : rb;
        hipLaunchKernelGGL(fn, dim3(grid), dim3(SB), lds, s, d, grp);
        return hipGetLastError();
    }
    constexpr int TB = K >= 7 ? 512 : 256;
    auto fn = tile_kernel<T, TRACK, K, TB>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           max_lds_bytes() - (int)kStaticLdsReserve);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(fn, dim3(nblocks), dim3(TB), lds, s, d, grp);
    return hipGetLastError();
}

template <typename T, bool TRACK>
static hipError_t launch_tile_k(const TilePassDesc *d, const TileGroups &grp, int k, size_t lds, hipStream_t s) {
    switch (k) {
    case 4: return launch_tile_t<T, TRACK, 4>(d, grp, lds, s);
    case 5: return launch_tile_t<T, TRACK, 5>(d, grp, lds, s);
    case 6: return launch_tile_t<T, TRACK, 6>(d, grp, lds, s);
    default: return launch_tile_t<T, TRACK, 7>(d, grp, lds, s);
    }
}

hipError_t launch_tile_pass(const TilePassDesc *d_descs, const TileGroups &grp, int k, int dtype_bytes, bool track,
                            hipStream_t s) {
    if (grp.ngroups <= 0 || grp.first_block[grp.ngroups] <= 0) return hipSuccess;
    if (k < 4 || k > 7) return hipErrorInvalidValue;
    const size_t lds = resident_lds_bytes(k, dtype_bytes, track);
    if (dtype_bytes == 8)
        return track ? launch_tile_k<double, true>(d_descs, grp, k, lds, s)
                     : launch_tile_k<double, false>(d_descs, grp, k, lds, s);
    return track ? launch_tile_k<float, true>(d_descs, grp, k, lds, s)
                 : launch_tile_k<float, false>(d_descs, grp, k, lds, s);
}

template <int K, int BLOCK>
static hipError_t launch_grad_t(const GradPassDesc *d, int ntiles, hipStream_t s) {
    auto fn = grad_kernel<K, BLOCK>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           max_lds_bytes() - (int)kStaticLdsReserve);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const size_t lds = 2 * sizeof(double) * ((size_t)1 << (2 * K));
    hipLaunchKernelGGL(fn, dim3(ntiles), dim3(BLOCK), lds, s, d);
    return hipGetLastError();
}

hipError_t launch_grad_pass(const GradPassDesc *d_desc, int ntiles, int k, hipStream_t s) {
    switch (k) {
    case 1: return launch_grad_t<1, 64>(d_desc, ntiles, s);
    case 2: return launch_grad_t<2, 64>(d_desc, ntiles, s);
    case 3: return launch_grad_t<3, 64>(d_desc, ntiles, s);
    case 4: return launch_grad_t<4, 64>(d_desc, ntiles, s);
    case 5: return launch_grad_t<5, 256>(d_desc, ntiles, s);
    case 6: return launch_grad_t<6, 256>(d_desc, ntiles, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_grad_init_state(double *r, int n, hipStream_t s) {
    const long long size = 1ll << (2 * n);
    const int grid = (int)((size + 255) / 256 < 4096 ? (size + 255) / 256 : 4096);
    hipLaunchKernelGGL(grad_init_state_kernel, dim3(grid), dim3(256), 0, s, r, n, size);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double *partials, int nslots, int ntiles, double *rot_grad, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((nslots + 255) / 256), dim3(256), 0, s, partials, nslots, ntiles,
                       rot_grad);
    return hipGetLastError();
}

hipError_t launch_grad_accumulate(const double *rot_grad, const int32_t *slot_param, int nslots, double *grad,
                                  int nparams, hipStream_t s) {
    hipLaunchKernelGGL(grad_accumulate_kernel, dim3(1), dim3(64), 0, s, rot_grad, slot_param, nslots, grad, nparams);
    return hipGetLastError();
}

hipError_t launch_copy_f64(const double *src, double *dst, long long count, hipStream_t s) {
    const int grid = (int)((count + 255) / 256 < 4096 ? (count + 255) / 256 : 4096);
    hipLaunchKernelGGL(copy_f64_n_kernel, dim3(grid), dim3(256), 0, s, src, dst, count);
    return hipGetLastError();
}

hipError_t launch_dense_init(void *coef, uint8_t *pres, int n, int dtype_bytes, const uint64_t *x,
                             const uint64_t *z, const double *c, int nterms, hipStream_t s, int count) {
    const long long size = 1ll << (2 * n);
    const long long total = size * count;
    const int grid = (int)((total + 255) / 256 < 8192 ? (total + 255) / 256 : 8192);
    if (dtype_bytes == 8) {
        hipLaunchKernelGGL(dense_fill_kernel<double>, dim3(grid), dim3(256), 0, s, (double *)coef, pres, total);
        hipLaunchKernelGGL(dense_scatter_kernel<double>, dim3(count), dim3(64), 0, s, (double *)coef, pres, n, x, z,
                           c, nterms, size);
    } else {
        hipLaunchKernelGGL(dense_fill_kernel<float>, dim3(grid), dim3(256), 0, s, (float *)coef, pres, total);
        hipLaunchKernelGGL(dense_scatter_kernel<float>, dim3(count), dim3(64), 0, s, (float *)coef, pres, n, x, z, c,
                           nterms, size);
    }
    return hipGetLastError();
}

hipError_t launch_dense_readout(const void *coef, int n, int dtype_bytes, double *out, hipStream_t s, int count) {
    const long long size = 1ll << (2 * n);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(dense_readout_kernel<double>, dim3(count), dim3(256), 0, s, (const double *)coef, n, out,
                           size);
    else
        hipLaunchKernelGGL(dense_readout_kernel<float>, dim3(count), dim3(256), 0, s, (const float *)coef, n, out,
                           size);
    return hipGetLastError();
}

hipError_t launch_dense_init_many(const DenseIODesc *d_descs, int nd, int max_n, int dtype_bytes, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    const long long size = 1ll << (2 * max_n);
    const int gx = (int)((size + 255) / 256 < 1024 ? (size + 255) / 256 : 1024);
    if (dtype_bytes == 8) {
        hipLaunchKernelGGL(many_fill_kernel<double>, dim3(gx, nd), dim3(256), 0, s, d_descs);
        hipLaunchKernelGGL(many_scatter_kernel<double>, dim3(nd), dim3(64), 0, s, d_descs);
    } else {
        hipLaunchKernelGGL(many_fill_kernel<float>, dim3(gx, nd), dim3(256), 0, s, d_descs);
        hipLaunchKernelGGL(many_scatter_kernel<float>, dim3(nd), dim3(64), 0, s, d_descs);
    }
    return hipGetLastError();
}

hipError_t launch_dense_readout_many(const DenseIODesc *d_descs, int nd, int dtype_bytes, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(many_readout_kernel<double>, dim3(nd), dim3(256), 0, s, d_descs);
    else
        hipLaunchKernelGGL(many_readout_kernel<float>, dim3(nd), dim3(256), 0, s, d_descs);
    return hipGetLastError();
}

hipError_t launch_dense_count(const uint8_t *pres, int n, unsigned long long *out, hipStream_t s) {
    const long long size = 1ll << (2 * n);
    const int grid = (int)((size + 255) / 256 < 2048 ? (size + 255) / 256 : 2048);
    hipLaunchKernelGGL(dense_count_kernel, dim3(grid), dim3(256), 0, s, pres, size, out);
    return hipGetLastError();
}

hipError_t launch_dense_compact(const void *coef, const uint8_t *pres, int n, int dtype_bytes, uint64_t *x,
                                uint64_t *z, double *c, unsigned long long *count, int *block_counts,
                                unsigned long long *, int *, hipStream_t s) {
    const long long size = 1ll << (2 * n);
    const int nb = (int)((size + CMP_CHUNK - 1) / CMP_CHUNK);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(compact_count_kernel<double>, dim3(nb), dim3(256), 0, s, (const double *)coef, pres, size,
                           block_counts);
    else
        hipLaunchKernelGGL(compact_count_kernel<float>, dim3(nb), dim3(256), 0, s, (const float *)coef, pres, size,
                           block_counts);
    hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(64), 0, s, block_counts, nb, count);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(compact_write_kernel<double>, dim3(nb), dim3(256), 0, s, (const double *)coef, pres, size,
                           n, block_counts, x, z, c);
    else
        hipLaunchKernelGGL(compact_write_kernel<float>, dim3(nb), dim3(256), 0, s, (const float *)coef, pres, size, n,
                           block_counts, x, z, c);
    return hipGetLastError();
}

}  // namespace pp
