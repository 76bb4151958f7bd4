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
#include "pp_device.h"

namespace pp {

// Bank swizzle for 8-byte LDS words: XOR the low 4 index bits with a
// function of bits 4-5.  It keeps every 16-slot block in place (so tiles
// smaller than 16 slots are unaffected) and spreads the three access
// patterns used below (quads on digit 0, on digit 1, and on digits >= 2)
// over distinct banks.
__device__ __forceinline__ int sw(int i) { return i ^ (((i >> 4) & 3) * 5); }

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

template <int BLOCK>
__device__ double block_sum_d(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double tot = 0.0;
    for (int i = 0; i < BLOCK / 64; ++i) tot += red[i];
    return tot;
}

template <int BLOCK>
__device__ long long block_sum_i(long long v, long long *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    long long tot = 0;
    for (int i = 0; i < BLOCK / 64; ++i) tot += red[i];
    return tot;
}

// ----------------------------------------------------------------- U1 op
// Quad u of digit a: the slots base + d * 4^a, d = 0..3, with base the index
// u with a zero digit inserted at position a.  Returns the number of
// strings created (tracked runs only).
template <typename T, bool TRACK>
__device__ __forceinline__ int u1_apply(T *lc, uint8_t *lp, int k, int a, const double *__restrict__ M,
                                        unsigned smask, int tid, int nthr) {
    const int nq = 1 << (2 * (k - 1));
    const int sh = 2 * a;
    const int lowmask = (1 << sh) - 1;
    const double m00 = M[0], m01 = M[1], m02 = M[2];
    const double m10 = M[3], m11 = M[4], m12 = M[5];
    const double m20 = M[6], m21 = M[7], m22 = M[8];
    int delta = 0;
    for (int u = tid; u < nq; u += nthr) {
        const int base = ((u & ~lowmask) << 2) | (u & lowmask);
        const int iX = base | (1 << sh), iZ = base | (2 << sh), iY = base | (3 << sh);
        const double cx = lds_ld(lc, iX), cy = lds_ld(lc, iY), cz = lds_ld(lc, iZ);
        lds_st(lc, iX, m00 * cx + m01 * cy + m02 * cz);
        lds_st(lc, iY, m10 * cx + m11 * cy + m12 * cz);
        lds_st(lc, iZ, m20 * cx + m21 * cy + m22 * cz);
        if (TRACK) {
            const unsigned old = (unsigned)lp[sw(iX)] | ((unsigned)lp[sw(iY)] << 1) | ((unsigned)lp[sw(iZ)] << 2);
            unsigned nw = 0;
#pragma unroll
            for (int r = 0; r < 3; ++r)
                if ((smask >> (3 * r)) & 7u & old) nw |= 1u << r;
            lp[sw(iX)] = (uint8_t)(nw & 1u);
            lp[sw(iY)] = (uint8_t)((nw >> 1) & 1u);
            lp[sw(iZ)] = (uint8_t)((nw >> 2) & 1u);
            delta += __popc(nw) - __popc(old);
        }
    }
    return delta;
}

// ----------------------------------------------------------------- CX op
// Group u of digits (a = control, b = target): the 16 slots base + dc*4^a +
// dt*4^b.  CX conjugation maps (xc, zc, xt, zt) to (xc, zc^zt, xt^xc, zt)
// with a sign flip iff xc & zt & !(xt ^ zc); the map is an involution, so
// the 12 moving slots form 6 signed swaps.
template <typename T, bool TRACK>
__device__ __forceinline__ void cx_apply(T *lc, uint8_t *lp, int k, int a, int b, int tid, int nthr) {
    const int ng = 1 << (2 * (k - 2));
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int mlo = (1 << (2 * lo)) - 1, mhi = (1 << (2 * hi)) - 1;
    const int sa = 2 * a, sb = 2 * b;
    for (int u = tid; u < ng; u += nthr) {
        int v = ((u & ~mlo) << 2) | (u & mlo);
        v = ((v & ~mhi) << 2) | (v & mhi);
#pragma unroll
        for (int dc = 0; dc < 4; ++dc) {
#pragma unroll
            for (int dt = 0; dt < 4; ++dt) {
                const int xc = dc & 1, zc = dc >> 1, xt = dt & 1, zt = dt >> 1;
                const int dc2 = xc | ((zc ^ zt) << 1), dt2 = (xt ^ xc) | (zt << 1);
                if (dc2 * 4 + dt2 > dc * 4 + dt) {
                    const bool neg = xc & zt & ((xt ^ zc) ^ 1);
                    const int i1 = v | (dc << sa) | (dt << sb);
                    const int i2 = v | (dc2 << sa) | (dt2 << sb);
                    const double v1 = lds_ld(lc, i1), v2 = lds_ld(lc, i2);
                    lds_st(lc, i1, neg ? -v2 : v2);
                    lds_st(lc, i2, neg ? -v1 : v1);
                    if (TRACK) {
                        const uint8_t p1 = lp[sw(i1)], p2 = lp[sw(i2)];
                        lp[sw(i1)] = p2;
                        lp[sw(i2)] = p1;
                    }
                }
            }
        }
    }
}

// Applies ops [o0, o1) to an LDS tile of 4^k slots.  For tracked runs it
// accumulates term updates: every op adds ngates * (strings in the tile
// before it), and U1 ops that can create strings update that count.
template <typename T, bool TRACK, int BLOCK>
__device__ void run_ops(T *lc, uint8_t *lp, int k, const DOp *__restrict__ ops, const double *__restrict__ maps,
                        int o0, int o1, long long &tcount, long long &updates, long long *redi) {
    const int tid = threadIdx.x;
    for (int o = o0; o < o1; ++o) {
        const DOp op = ops[o];
        if (op.kind == DOP_U1) {
            const int delta = u1_apply<T, TRACK>(lc, lp, k, op.a, maps + 9ull * op.map, op.smask, tid, BLOCK);
            if (TRACK) {
                updates += tcount * op.ngates;
                if (!op.perm) tcount += block_sum_i<BLOCK>(delta, redi);
            }
        } else {
            cx_apply<T, TRACK>(lc, lp, k, op.a, op.b, tid, BLOCK);
            if (TRACK) updates += tcount * op.ngates;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- resident kernel
// One workgroup runs one whole circuit (n <= 7) in LDS: builds the
// observable, applies every op, reads out <O> and optionally stores the
// final weights / presence for pp_get_terms.
template <typename T, bool TRACK, int BLOCK>
__global__ __launch_bounds__(BLOCK) void resident_kernel(const ResidentDesc *__restrict__ descs) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double redd[BLOCK / 64];
    __shared__ long long redi[BLOCK / 64];
    const ResidentDesc &d = descs[blockIdx.x];
    const int n = d.n;
    const int size = 1 << (2 * n);
    T *lc = reinterpret_cast<T *>(smem);
    uint8_t *lp = smem + (size_t)size * sizeof(T);
    const int tid = threadIdx.x;

    for (int i = tid; i < size; i += BLOCK) {
        lc[i] = (T)0;
        if (TRACK) lp[i] = 0;
    }
    __syncthreads();
    if (tid == 0) {
        for (int t = 0; t < d.nterms; ++t) {
            const int s = (int)morton_slot(d.obs_x[t], d.obs_z[t], n);
            lc[sw(s)] = (T)((double)lc[sw(s)] + d.obs_c[t]);
            if (TRACK) lp[sw(s)] = 1;
        }
    }
    __syncthreads();

    long long tcount = 0, updates = 0;
    if (TRACK) {
        long long mine = 0;
        for (int i = tid; i < size; i += BLOCK) mine += lp[i];
        tcount = block_sum_i<BLOCK>(mine, redi);
    }
    run_ops<T, TRACK, BLOCK>(lc, lp, n, d.ops, d.maps, 0, d.nops, tcount, updates, redi);

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
template <typename T, bool TRACK, int BLOCK>
__global__ __launch_bounds__(BLOCK) void tile_kernel(const TilePassDesc *__restrict__ descs, int ndescs) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long redi[BLOCK / 64];
    int lo = 0, hi = ndescs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].tile_begin <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const TilePassDesc &d = descs[lo];
    const long long tile = (long long)blockIdx.x - d.tile_begin;
    const int k = d.k, n = d.n;
    const int size = 1 << (2 * k);
    T *lc = reinterpret_cast<T *>(smem);
    uint8_t *lp = smem + (size_t)size * sizeof(T);
    const int tid = threadIdx.x;

    unsigned inmask = 0;
    for (int j = 0; j < k; ++j) inmask |= 1u << d.qubit[j];
    long long base = 0;
    {
        long long t = tile;
        for (int q = 0; q < n; ++q) {
            if ((inmask >> q) & 1u) continue;
            base |= (t & 3ll) << (2 * q);
            t >>= 2;
        }
    }
    int jlow = 0;
    while (jlow < k && d.qubit[jlow] == jlow) ++jlow;
    const int lowmask = (1 << (2 * jlow)) - 1;

    T *g = reinterpret_cast<T *>(d.coef);
    for (int i = tid; i < size; i += BLOCK) {
        long long gi = base | (i & lowmask);
        for (int j = jlow; j < k; ++j) gi |= (long long)((i >> (2 * j)) & 3) << (2 * d.qubit[j]);
        lc[sw(i)] = g[gi];
        if (TRACK) lp[sw(i)] = d.pres[gi];
    }
    __syncthreads();

    long long tcount = 0, updates = 0;
    if (TRACK) {
        long long mine = 0;
        for (int i = tid; i < size; i += BLOCK) mine += lp[i];
        tcount = block_sum_i<BLOCK>(mine, redi);
    }
    run_ops<T, TRACK, BLOCK>(lc, lp, k, d.ops, d.maps, d.op_begin, d.op_end, tcount, updates, redi);

    for (int i = tid; i < size; i += BLOCK) {
        long long gi = base | (i & lowmask);
        for (int j = jlow; j < k; ++j) gi |= (long long)((i >> (2 * j)) & 3) << (2 * d.qubit[j]);
        g[gi] = lc[sw(i)];
        if (TRACK) d.pres[gi] = lp[sw(i)];
    }
    if (TRACK && tid == 0 && updates) atomicAdd(d.counters, (unsigned long long)updates);
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

__global__ void compose_kernel(const ComposeDesc *__restrict__ descs) {
    const ComposeDesc &d = descs[blockIdx.x];
    for (int i = threadIdx.x; i < d.nmaps; i += blockDim.x) {
        double M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        for (int r = d.roff[i]; r < d.roff[i + 1]; ++r) {
            const int op = d.rop[r];
            const double th = op >= 3 ? d.theta[d.rparam[r]] : 0.0;
            double G[9], P[9];
            gate_matrix(op, th, G);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    P[3 * a + b] = G[3 * a] * M[b] + G[3 * a + 1] * M[3 + b] + G[3 * a + 2] * M[6 + b];
            for (int t = 0; t < 9; ++t) M[t] = P[t];
        }
        for (int t = 0; t < 9; ++t) d.maps[9ull * i + t] = M[t];
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

// Sequential so that repeated strings are summed in input order.
template <typename T>
__global__ void dense_scatter_kernel(T *coef, uint8_t *pres, int n, const uint64_t *x, const uint64_t *z,
                                     const double *c, int nterms) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int t = 0; t < nterms; ++t) {
        const long long s = morton_slot(x[t], z[t], n);
        coef[s] = (T)((double)coef[s] + c[t]);
        if (pres) pres[s] = 1;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void dense_readout_kernel(const T *coef, int n, double *out) {
    __shared__ double redd[4];
    double part = 0.0;
    for (long long j = threadIdx.x; j < (1ll << n); j += 256) part += (double)coef[zonly_slot(j, n)];
    const double tot = block_sum_d<256>(part, redd);
    if (threadIdx.x == 0) *out = tot;
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

__global__ __launch_bounds__(256) void compact_count_kernel(const uint8_t *pres, long long size, int *counts) {
    __shared__ long long redi[4];
    const long long b0 = (long long)blockIdx.x * CMP_CHUNK;
    long long mine = 0;
    for (int i = threadIdx.x; i < CMP_CHUNK; i += 256)
        if (b0 + i < size) mine += pres[b0 + i];
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
    __syncthreads();
    for (int r = 0; r < CMP_CHUNK; r += 256) {
        const long long i = b0 + r + threadIdx.x;
        const bool p = i < size && pres[i];
        const unsigned long long bal = __ballot(p);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[w] = __popcll(bal);
        __syncthreads();
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
        __syncthreads();
        if (threadIdx.x == 0) running += wcount[0] + wcount[1] + wcount[2] + wcount[3];
        __syncthreads();
    }
}

// ------------------------------------------------------------ launchers
int max_lds_bytes() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return v;
}

size_t resident_lds_bytes(int n, int dtype_bytes, bool track) {
    const size_t size = (size_t)1 << (2 * n);
    return size * (size_t)dtype_bytes + (track ? size : 0);
}

hipError_t launch_compose(const ComposeDesc *d_descs, int ndescs, hipStream_t s) {
    if (ndescs <= 0) return hipSuccess;
    hipLaunchKernelGGL(compose_kernel, dim3(ndescs), dim3(256), 0, s, d_descs);
    return hipGetLastError();
}

template <typename T, bool TRACK, int BLOCK>
static hipError_t launch_res_t(const ResidentDesc *d, int nd, size_t lds, hipStream_t s) {
    auto fn = resident_kernel<T, TRACK, BLOCK>;
    hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(nd), dim3(BLOCK), lds, s, d);
    return hipGetLastError();
}

template <typename T, bool TRACK>
static hipError_t launch_res_b(const ResidentDesc *d, int nd, int n, size_t lds, hipStream_t s) {
    if (n <= 3) return launch_res_t<T, TRACK, 64>(d, nd, lds, s);
    if (n <= 5) return launch_res_t<T, TRACK, 256>(d, nd, lds, s);
    return launch_res_t<T, TRACK, 512>(d, nd, lds, s);
}

hipError_t launch_resident(const ResidentDesc *d_descs, int ndescs, int n, int dtype_bytes, bool track,
                           hipStream_t s) {
    if (ndescs <= 0) return hipSuccess;
    const size_t lds = resident_lds_bytes(n, dtype_bytes, track);
    if (dtype_bytes == 8)
        return track ? launch_res_b<double, true>(d_descs, ndescs, n, lds, s)
                     : launch_res_b<double, false>(d_descs, ndescs, n, lds, s);
    return track ? launch_res_b<float, true>(d_descs, ndescs, n, lds, s)
                 : launch_res_b<float, false>(d_descs, ndescs, n, lds, s);
}

template <typename T, bool TRACK, int BLOCK>
static hipError_t launch_tile_t(const TilePassDesc *d, int nd, int nblocks, size_t lds, hipStream_t s) {
    auto fn = tile_kernel<T, TRACK, BLOCK>;
    hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(nblocks), dim3(BLOCK), lds, s, d, nd);
    return hipGetLastError();
}

hipError_t launch_tile_pass(const TilePassDesc *d_descs, int ndescs, int nblocks, int k, int dtype_bytes,
                            bool track, hipStream_t s) {
    if (ndescs <= 0 || nblocks <= 0) return hipSuccess;
    const size_t lds = resident_lds_bytes(k, dtype_bytes, track);
    if (dtype_bytes == 8)
        return track ? launch_tile_t<double, true, 256>(d_descs, ndescs, nblocks, lds, s)
                     : launch_tile_t<double, false, 256>(d_descs, ndescs, nblocks, lds, s);
    return track ? launch_tile_t<float, true, 256>(d_descs, ndescs, nblocks, lds, s)
                 : launch_tile_t<float, false, 256>(d_descs, ndescs, nblocks, lds, s);
}

hipError_t launch_dense_init(void *coef, uint8_t *pres, int n, int dtype_bytes, const uint64_t *x,
                             const uint64_t *z, const double *c, int nterms, hipStream_t s) {
    const long long size = 1ll << (2 * n);
    const int grid = (int)((size + 255) / 256 < 4096 ? (size + 255) / 256 : 4096);
    if (dtype_bytes == 8) {
        hipLaunchKernelGGL(dense_fill_kernel<double>, dim3(grid), dim3(256), 0, s, (double *)coef, pres, size);
        hipLaunchKernelGGL(dense_scatter_kernel<double>, dim3(1), dim3(64), 0, s, (double *)coef, pres, n, x, z, c,
                           nterms);
    } else {
        hipLaunchKernelGGL(dense_fill_kernel<float>, dim3(grid), dim3(256), 0, s, (float *)coef, pres, size);
        hipLaunchKernelGGL(dense_scatter_kernel<float>, dim3(1), dim3(64), 0, s, (float *)coef, pres, n, x, z, c,
                           nterms);
    }
    return hipGetLastError();
}

hipError_t launch_dense_readout(const void *coef, int n, int dtype_bytes, double *out, hipStream_t s) {
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(dense_readout_kernel<double>, dim3(1), dim3(256), 0, s, (const double *)coef, n, out);
    else
        hipLaunchKernelGGL(dense_readout_kernel<float>, dim3(1), dim3(256), 0, s, (const float *)coef, n, out);
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
    hipLaunchKernelGGL(compact_count_kernel, dim3(nb), dim3(256), 0, s, pres, size, block_counts);
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
