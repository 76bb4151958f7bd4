// Sparse engine of libpauliprop: an explicit list of weighted Pauli strings.
//
// Layout: struct of arrays x[cap], z[cap] (one 64-bit symplectic word per
// term each, bit q = qubit q, so n <= 64) and c[cap] (FP64 or FP32 weight),
// with the live count kept on the device.  One pass (Sec. IV-B: Map applies
// the operators in order, each one's output feeding the next) is
//   1. per term, in registers: a run of Clifford gates (H, S, CX as g^dag P g:
//      the H and S rows of Table I inverted and the CX list of Sec. III-C;
//      a Clifford maps a string to one string and may flip the sign);
//   2. the run's closing rotation R_sigma(theta): a string that anticommutes
//      with sigma keeps cos(theta) of its weight in place and appends a child
//      string sigma-flipped with +-sin(theta) (R rows of Table I, Example 1);
//      children are appended in term order by wave-ballot compaction with a
//      reduce-then-scan over blocks (no atomics, so the order is fixed);
//   3. merging of equal strings (reduce(), eq. (7), Examples 3-4): LSD radix
//      sort on the 2n-bit key (z, x) with LDS-staged stable tiles, then a
//      segmented FP64 sum that keeps one string per key, zero sums included.
// Every step runs three-phase (count, scan, write) so results are
// reproducible bit for bit.
#include "pp_device.h"

namespace pp {

constexpr int SP_BLOCK = 256;
constexpr int SP_ITEMS = 8;
constexpr int SP_TILE = SP_BLOCK * SP_ITEMS;  // 2048 terms per block
constexpr int SP_GRID = 2048;  // cap on the workgroups of a tile kernel

template <typename T>
__device__ __forceinline__ double ldc(const void *p, long long i) { return (double)((const T *)p)[i]; }
template <typename T>
__device__ __forceinline__ void stc(void *p, long long i, double v) { ((T *)p)[i] = (T)v; }

// ------------------------------------------------ Clifford run + rotation
__device__ __forceinline__ void clifford_apply(uint64_t &x, uint64_t &z, unsigned &neg, const uint32_t *__restrict__ codes,
                                               int g0, int g1) {
    for (int g = g0; g < g1; ++g) {
        const uint32_t code = codes[g];
        const int op = code & 0xff, a = (code >> 8) & 0xff, b = (code >> 16) & 0xff;
        const unsigned xa = (unsigned)(x >> a) & 1u, za = (unsigned)(z >> a) & 1u;
        if (op == 0) {  // H: X <-> Z, Y -> -Y
            neg ^= xa & za;
            const uint64_t f = (uint64_t)(xa ^ za) << a;
            x ^= f;
            z ^= f;
        } else if (op == 1) {  // S^dag . S: X -> -Y, Y -> X
            neg ^= xa & (za ^ 1u);
            z ^= (uint64_t)xa << a;
        } else {  // CX(a -> b): x_b ^= x_a, z_a ^= z_b, sign x_a z_b !(x_b ^ z_a)
            const unsigned xb = (unsigned)(x >> b) & 1u, zb = (unsigned)(z >> b) & 1u;
            neg ^= xa & zb & ((xb ^ za) ^ 1u);
            x ^= (uint64_t)xa << b;
            z ^= (uint64_t)zb << a;
        }
    }
}

// non-identity letters of a string
__device__ __forceinline__ int pauli_weight(uint64_t x, uint64_t z) { return __popcll(x | z); }

// sum over a SP_BLOCK workgroup in a fixed order (lanes, then waves)
__device__ __forceinline__ double block_sum_d(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < SP_BLOCK / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// anticommutation with sigma on qubit q, the child's flipped bits and sign
__device__ __forceinline__ bool rot_child(int op, int q, uint64_t x, uint64_t z, uint64_t &fx, uint64_t &fz, double &sg) {
    const unsigned xb = (unsigned)(x >> q) & 1u, zb = (unsigned)(z >> q) & 1u;
    const uint64_t bit = 1ull << q;
    if (op == 3) {  // RX: Y -> cY - sZ, Z -> cZ + sY
        fx = bit; fz = 0; sg = xb ? -1.0 : 1.0;
        return zb;
    }
    if (op == 4) {  // RY: X -> cX + sZ, Z -> cZ - sX
        fx = bit; fz = bit; sg = xb ? 1.0 : -1.0;
        return xb ^ zb;
    }
    // RZ: X -> cX - sY, Y -> cY + sX
    fx = 0; fz = bit; sg = zb ? 1.0 : -1.0;
    return xb;
}

// Every kernel below covers only the live tiles: the grid is capped at
// SP_GRID workgroups and each workgroup strides over tiles, the live count
// being read from device memory, so a small term set costs a small pass.
__device__ __forceinline__ long long live_tiles(long long T) { return (T + SP_TILE - 1) / SP_TILE; }

// phase 1: count anticommuting terms per tile
__global__ __launch_bounds__(SP_BLOCK) void pass_count_kernel(const uint64_t *__restrict__ x, const uint64_t *__restrict__ z,
                                                             const long long *__restrict__ count,
                                                             const uint32_t *__restrict__ codes, SparsePassDesc p,
                                                             int *__restrict__ bcounts, int max_weight) {
    __shared__ int red[SP_BLOCK / 64];
    const long long T = count[0];
    const long long L = live_tiles(T);
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        const long long b0 = t * SP_TILE;
        int mine = 0;
        if (p.rot_op >= 3) {
            for (int it = 0; it < SP_ITEMS; ++it) {
                const long long i = b0 + it * SP_BLOCK + threadIdx.x;
                if (i < T) {
                    uint64_t xx = x[i], zz = z[i];
                    unsigned neg = 0;
                    clifford_apply(xx, zz, neg, codes, p.g_begin, p.g_end);
                    uint64_t fx, fz;
                    double sg;
                    mine += (rot_child(p.rot_op, p.rot_q, xx, zz, fx, fz, sg) &&
                             pauli_weight(xx ^ fx, zz ^ fz) <= max_weight)
                                ? 1
                                : 0;
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mine;
        __syncthreads();
        if (threadIdx.x == 0) {
            int s = 0;
            for (int w = 0; w < SP_BLOCK / 64; ++w) s += red[w];
            bcounts[t] = s;
        }
        __syncthreads();
    }
}

// Exclusive scan, in place, of a[0, len) with len = mult * (tiles of `tile`
// terms that count[0] terms fill).  SCAN_BLOCKS workgroups each own one contiguous chunk: the first
// kernel sums every chunk, the second adds to each chunk the sums of the
// chunks before it and scans it; the last workgroup leaves the grand total.
constexpr int SCAN_BLOCKS = 256;

__device__ __forceinline__ void scan_chunk(long long len, long long &lo, long long &hi) {
    const long long chunk = (len + SCAN_BLOCKS - 1) / SCAN_BLOCKS;
    lo = (long long)blockIdx.x * chunk;
    hi = lo + chunk < len ? lo + chunk : len;
}

__device__ __forceinline__ long long block_sum_1024(long long v, long long *wsum) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = 0;
    for (int u = 0; u < 16; ++u) t += wsum[u];
    __syncthreads();
    return t;
}

template <typename V>
__global__ __launch_bounds__(1024) void scan_reduce_kernel(const V *__restrict__ a, const long long *__restrict__ count,
                                                          int mult, int tile, long long *__restrict__ bsum) {
    __shared__ long long wsum[16];
    long long lo, hi;
    scan_chunk(mult * ((count[0] + tile - 1) / tile), lo, hi);
    long long s = 0;
    for (long long i = lo + threadIdx.x; i < hi; i += 1024) s += (long long)a[i];
    s = block_sum_1024(s, wsum);
    if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

template <typename V>
__global__ __launch_bounds__(1024) void scan_apply_kernel(V *__restrict__ a, const long long *__restrict__ count, int mult,
                                                         int tile, const long long *__restrict__ bsum,
                                                         long long *__restrict__ total) {
    __shared__ long long wsum[16];
    __shared__ long long carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    long long lo, hi;
    scan_chunk(mult * ((count[0] + tile - 1) / tile), lo, hi);
    const long long before = block_sum_1024(tid < (int)blockIdx.x ? bsum[tid] : 0, wsum);
    if (tid == 0) carry = before;
    __syncthreads();
    for (long long b0 = lo; b0 < hi; b0 += 1024) {
        const long long i = b0 + tid;
        const long long v = i < hi ? (long long)a[i] : 0;
        long long inc = v;
        for (int off = 1; off < 64; off <<= 1) {
            const long long o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        long long pre = carry;
        for (int u = 0; u < w; ++u) pre += wsum[u];
        if (i < hi) a[i] = (V)(pre + inc - v);
        __syncthreads();
        if (tid == 0) {
            long long t = 0;
            for (int u = 0; u < 16; ++u) t += wsum[u];
            carry += t;
        }
        __syncthreads();
    }
    if (blockIdx.x == SCAN_BLOCKS - 1 && tid == 0) *total = carry;
}

// phase 2 tail: appends the children after the live terms, flags overflow,
// and counts term updates
__global__ void pass_finalize_kernel(long long *__restrict__ count, const long long *__restrict__ total, long long cap2,
                                     unsigned long long *__restrict__ updates, int ngates,
                                     long long *__restrict__ child_base) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const long long T = count[0];
    *updates += (unsigned long long)T * (unsigned long long)ngates;
    child_base[0] = T;
    long long nt = T + *total;
    if (nt > cap2) {
        count[1] = 1;
        nt = cap2;
    }
    count[0] = nt;
}

// phase 3: apply the run, rescale parents in place, write children in order
template <typename T>
__global__ __launch_bounds__(SP_BLOCK) void pass_write_kernel(uint64_t *__restrict__ x, uint64_t *__restrict__ z, void *c,
                                                             const long long *__restrict__ child_base, long long cap2,
                                                             const uint32_t *__restrict__ codes, SparsePassDesc p,
                                                             const double *__restrict__ theta,
                                                             const int *__restrict__ boffs, int max_weight,
                                                             double *__restrict__ dropped) {
    __shared__ int wcnt[SP_BLOCK / 64];
    __shared__ int running;
    __shared__ double redd[SP_BLOCK / 64];
    const long long nlive = child_base[0];
    const long long L = live_tiles(nlive);
    if ((long long)blockIdx.x >= L) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double cs = 1.0, sn = 0.0;
    const bool rot = p.rot_op >= 3;
    if (rot) sincos(theta[p.rot_param], &sn, &cs);
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        const long long b0 = t * SP_TILE;
        if (threadIdx.x == 0) running = boffs[t];
        __syncthreads();
        double lost = 0.0;  // weight of children above max_weight (truncation)
        for (int it = 0; it < SP_ITEMS; ++it) {
            const long long i = b0 + it * SP_BLOCK + threadIdx.x;
            const bool live = i < nlive;
            uint64_t xx = 0, zz = 0, fx = 0, fz = 0;
            double cc = 0.0, sg = 1.0;
            bool anti = false, split = false;
            if (live) {
                xx = x[i];
                zz = z[i];
                cc = ldc<T>(c, i);
                unsigned neg = 0;
                clifford_apply(xx, zz, neg, codes, p.g_begin, p.g_end);
                if (neg) cc = -cc;
                if (rot) split = rot_child(p.rot_op, p.rot_q, xx, zz, fx, fz, sg);
                anti = split && pauli_weight(xx ^ fx, zz ^ fz) <= max_weight;
                if (split && !anti) lost += fabs(cc * sg * sn);
            }
            const unsigned long long bal = __ballot(anti);
            const int below = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) wcnt[w] = __popcll(bal);
            __syncthreads();
            int off = running;
            for (int u = 0; u < w; ++u) off += wcnt[u];
            if (live) {
                x[i] = xx;
                z[i] = zz;
                stc<T>(c, i, split ? cc * cs : cc);
                if (anti) {
                    const long long j = nlive + off + below;
                    if (j < cap2) {
                        x[j] = xx ^ fx;
                        z[j] = zz ^ fz;
                        stc<T>(c, j, cc * sg * sn);
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int s = 0;
                for (int u = 0; u < SP_BLOCK / 64; ++u) s += wcnt[u];
                running += s;
            }
            __syncthreads();
        }
        if (dropped) {
            const double tl = block_sum_d(lost, redd);
            if (threadIdx.x == 0) dropped[t] = tl;
        }
    }
}

// Adds the per-tile dropped weights of the tiles of the kernel before
// (live_tiles of *cnt) to dropped[total_at], in a fixed order.
__global__ __launch_bounds__(SP_BLOCK) void trunc_total_kernel(double *__restrict__ dropped,
                                                              const long long *__restrict__ cnt, long long total_at) {
    __shared__ double redd[SP_BLOCK / 64];
    const long long L = live_tiles(cnt[0]);
    double v = 0.0;
    for (long long t = threadIdx.x; t < L; t += SP_BLOCK) v += dropped[t];
    v = block_sum_d(v, redd);
    if (threadIdx.x == 0) dropped[total_at] += v;
}

// ---------------------------------------------------------- radix sort
// Key = (z << n) | x as a 2n-bit integer (canonical order: by z, then x).
// The sort's shape is a runtime choice (pp_tune_set): BITS key bits per
// pass with one thread per digit value (2^BITS threads), ITEMS terms per
// thread, so a tile holds 2^BITS x ITEMS terms.  Every shape is a stable LSD
// sort on the same key, so every shape gives the same order.
template <int BITS>
__device__ __forceinline__ unsigned key_digit(uint64_t x, uint64_t z, int n, int s) {
    uint64_t v;
    if (s >= n) v = z >> (s - n);
    else if (s + BITS <= n) v = x >> s;
    else v = (x >> s) | (z << (n - s));
    return (unsigned)(v & ((1u << BITS) - 1));
}

// Histograms are digit-major over the live tiles: hist[d * L + tile], so an
// exclusive scan of hist[0, 2^BITS * L) gives every (digit, tile) its output
// position.
template <int BITS, int ITEMS>
__global__ __launch_bounds__(1 << BITS) void sort_hist_kernel(const uint64_t *__restrict__ x, const uint64_t *__restrict__ z,
                                                              const long long *__restrict__ count, int n, int shift,
                                                              unsigned *__restrict__ hist) {
    constexpr int RX = 1 << BITS, BLOCK = RX, TILE = BLOCK * ITEMS;
    __shared__ unsigned h[RX];
    const long long T = count[0];
    const long long L = (T + TILE - 1) / TILE;
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        h[threadIdx.x] = 0;
        __syncthreads();
        const long long b0 = t * TILE;
        for (int it = 0; it < ITEMS; ++it) {
            const long long i = b0 + it * BLOCK + threadIdx.x;
            if (i < T) atomicAdd(&h[key_digit<BITS>(x[i], z[i], n, shift)], 1u);
        }
        __syncthreads();
        hist[(long long)threadIdx.x * L + t] = h[threadIdx.x];
        __syncthreads();
    }
}

// Stable scatter of one tile.  Wave w owns the contiguous sub-tile
// [w*64*ITEMS, (w+1)*64*ITEMS) and walks it in chunks of 64; lanes with
// equal digits are matched with BITS ballots, so the rank of a term is
// (terms of its digit in earlier waves) + (earlier chunks of its wave) +
// (lower lanes of its chunk).  Terms are staged in LDS in sorted order and
// written out so that each digit's run leaves the workgroup contiguously.
template <typename T, int BITS, int ITEMS>
__global__ __launch_bounds__(1 << BITS) void sort_scatter_kernel(const uint64_t *__restrict__ x,
                                                                 const uint64_t *__restrict__ z, const void *c,
                                                                 uint64_t *__restrict__ xo, uint64_t *__restrict__ zo,
                                                                 void *co, const long long *__restrict__ count, int n,
                                                                 int shift, const unsigned *__restrict__ hist) {
    constexpr int RX = 1 << BITS, BLOCK = RX, TILE = BLOCK * ITEMS, WAVES = BLOCK / 64;
    static_assert(BLOCK >= 64, "at least one full wave");
    __shared__ unsigned whist[WAVES][RX];
    __shared__ unsigned tpre[RX];
    __shared__ unsigned goff[RX];
    __shared__ uint64_t sx[TILE];
    __shared__ uint64_t sz[TILE];
    __shared__ T sc[TILE];
    const long long Tn = count[0];
    const long long L = (Tn + TILE - 1) / TILE;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        const long long b0 = t * TILE;
        {
            const int d = threadIdx.x;
            for (int v = 0; v < WAVES; ++v) whist[v][d] = 0;
            goff[d] = hist[(long long)d * L + t];
        }
        __syncthreads();

        uint64_t rx[ITEMS], rz[ITEMS];
        T rc[ITEMS];
        unsigned rd[ITEMS], rr[ITEMS];
        for (int j = 0; j < ITEMS; ++j) {
            const long long i = b0 + (long long)w * (ITEMS * 64) + j * 64 + lane;
            const bool live = i < Tn;
            rx[j] = live ? x[i] : 0;
            rz[j] = live ? z[i] : 0;
            rc[j] = live ? ((const T *)c)[i] : (T)0;
            const unsigned d = key_digit<BITS>(rx[j], rz[j], n, shift);
            unsigned long long peers = __ballot(live);
            for (int bt = 0; bt < BITS; ++bt) {
                const unsigned long long bb = __ballot((d >> bt) & 1u);
                peers &= ((d >> bt) & 1u) ? bb : ~bb;
            }
            const unsigned before = whist[w][d];
            __builtin_amdgcn_wave_barrier();
            const int rank = __popcll(peers & lt);
            if (live && rank == 0) whist[w][d] = before + (unsigned)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            rd[j] = live ? d : RX;
            rr[j] = before + (unsigned)rank;
        }
        __syncthreads();
        // per digit: exclusive prefix over waves, then an exclusive scan of the
        // tile's digit totals (thread d owns digit d)
        {
            const int d = threadIdx.x;
            unsigned run = 0;
            for (int v = 0; v < WAVES; ++v) {
                const unsigned cnt = whist[v][d];
                whist[v][d] = run;
                run += cnt;
            }
            unsigned inc = run;
            for (int off = 1; off < 64; off <<= 1) {
                const unsigned o = __shfl_up(inc, off, 64);
                if (lane >= off) inc += o;
            }
            tpre[d] = inc;
            __syncthreads();
            unsigned add = 0;
            for (int v = 0; v < w; ++v) add += tpre[v * 64 + 63];
            __syncthreads();
            tpre[d] = add + inc - run;
        }
        __syncthreads();
        for (int j = 0; j < ITEMS; ++j) {
            if (rd[j] < RX) {
                const unsigned pos = tpre[rd[j]] + whist[w][rd[j]] + rr[j];
                sx[pos] = rx[j];
                sz[pos] = rz[j];
                sc[pos] = rc[j];
            }
        }
        __syncthreads();
        const int valid = (int)((Tn - b0) < TILE ? (Tn - b0) : TILE);
        for (int i = threadIdx.x; i < valid; i += BLOCK) {
            const unsigned d = key_digit<BITS>(sx[i], sz[i], n, shift);
            const long long g = (long long)goff[d] + (i - (long long)tpre[d]);
            xo[g] = sx[i];
            zo[g] = sz[i];
            ((T *)co)[g] = sc[i];
        }
        __syncthreads();
    }
}

// --------------------------------------------------------- segmented sum
__device__ __forceinline__ bool seg_head(const uint64_t *x, const uint64_t *z, long long i) {
    return i == 0 || x[i] != x[i - 1] || z[i] != z[i - 1];
}

// A merged string survives truncation if its weight and |sum| allow it
template <typename T>
__device__ __forceinline__ bool seg_keep(const uint64_t *x, const uint64_t *z, const void *c, long long i, long long nlive,
                                         int max_weight, double eps, double &sum) {
    double s = ldc<T>(c, i);
    for (long long j = i + 1; j < nlive && x[j] == x[i] && z[j] == z[i]; ++j) s += ldc<T>(c, j);
    sum = s;
    return pauli_weight(x[i], z[i]) <= max_weight && fabs(s) >= eps;
}

template <typename TW>
__global__ __launch_bounds__(SP_BLOCK) void seg_count_kernel(const uint64_t *__restrict__ x, const uint64_t *__restrict__ z,
                                                            const void *c, const long long *__restrict__ count,
                                                            int *__restrict__ bcounts, int trunc, int max_weight,
                                                            double eps) {
    __shared__ int red[SP_BLOCK / 64];
    const long long T = count[0];
    const long long L = live_tiles(T);
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        const long long b0 = t * SP_TILE;
        int mine = 0;
        for (int it = 0; it < SP_ITEMS; ++it) {
            const long long i = b0 + it * SP_BLOCK + threadIdx.x;
            if (i < T && seg_head(x, z, i)) {
                double s;
                if (!trunc || seg_keep<TW>(x, z, c, i, T, max_weight, eps, s)) ++mine;
            }
        }
        for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mine;
        __syncthreads();
        if (threadIdx.x == 0) {
            int s = 0;
            for (int w = 0; w < SP_BLOCK / 64; ++w) s += red[w];
            bcounts[t] = s;
        }
        __syncthreads();
    }
}

// the merged count replaces the live count; the old one stays for the write
__global__ void seg_finalize_kernel(long long *__restrict__ count, const long long *__restrict__ total,
                                    long long *__restrict__ old_count) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    old_count[0] = count[0];
    count[0] = *total;
}

template <typename T>
__global__ __launch_bounds__(SP_BLOCK) void seg_write_kernel(const uint64_t *__restrict__ x, const uint64_t *__restrict__ z,
                                                            const void *c, uint64_t *__restrict__ xo,
                                                            uint64_t *__restrict__ zo, void *co,
                                                            const long long *__restrict__ old_count,
                                                            const int *__restrict__ boffs, int trunc, int max_weight,
                                                            double eps, double *__restrict__ dropped) {
    __shared__ int wcnt[SP_BLOCK / 64];
    __shared__ int running;
    __shared__ double redd[SP_BLOCK / 64];
    const long long nlive = old_count[0];
    const long long L = live_tiles(nlive);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        const long long b0 = t * SP_TILE;
        if (threadIdx.x == 0) running = boffs[t];
        __syncthreads();
        double lost = 0.0;
        for (int it = 0; it < SP_ITEMS; ++it) {
            const long long i = b0 + it * SP_BLOCK + threadIdx.x;
            bool head = i < nlive && seg_head(x, z, i);
            double ts = 0.0;
            if (head && trunc && !seg_keep<T>(x, z, c, i, nlive, max_weight, eps, ts)) {
                lost += fabs(ts);
                head = false;
            }
            const unsigned long long bal = __ballot(head);
            const int below = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) wcnt[w] = __popcll(bal);
            __syncthreads();
            int off = running;
            for (int u = 0; u < w; ++u) off += wcnt[u];
            if (head) {
                double s = ldc<T>(c, i);
                for (long long j = i + 1; j < nlive && x[j] == x[i] && z[j] == z[i]; ++j) s += ldc<T>(c, j);
                const long long o = off + below;
                xo[o] = x[i];
                zo[o] = z[i];
                stc<T>(co, o, s);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int s = 0;
                for (int u = 0; u < SP_BLOCK / 64; ++u) s += wcnt[u];
                running += s;
            }
            __syncthreads();
        }
        if (trunc) {
            const double tl = block_sum_d(lost, redd);
            if (threadIdx.x == 0) dropped[t] = tl;
        }
    }
}

// -------------------------------------------------------------- readout
constexpr int RO_BLOCKS = 256;

template <typename T>
__global__ __launch_bounds__(256) void sp_readout_partial_kernel(const uint64_t *__restrict__ x, const void *c,
                                                                const long long *__restrict__ count,
                                                                double *__restrict__ partials) {
    __shared__ double red[4];
    const long long Tn = count[0];
    const long long per = (Tn + RO_BLOCKS - 1) / RO_BLOCKS;
    const long long lo = blockIdx.x * per, hi = lo + per < Tn ? lo + per : Tn;
    double s = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += 256)
        if (x[i] == 0) s += ldc<T>(c, i);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void sp_readout_final_kernel(const double *__restrict__ partials, const long long *__restrict__ count,
                                        double *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < RO_BLOCKS; ++b) s += partials[b];
    *out = count[1] ? __builtin_nan("") : s;
}

// ---------------------------------------------------------------- init
template <typename T>
__global__ void sp_init_kernel(uint64_t *x, uint64_t *z, void *c, long long *count, unsigned long long *updates,
                               const uint64_t *ox, const uint64_t *oz, const double *oc, int nterms,
                               double *dropped_total) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    if (dropped_total) *dropped_total = 0.0;
    for (int t = 0; t < nterms; ++t) {
        x[t] = ox[t];
        z[t] = oz[t];
        stc<T>(c, t, oc[t]);
    }
    count[0] = nterms;
    count[1] = 0;
    *updates = 0;
}

// ============================================================ Clifford frame
// The stored strings never see a Clifford gate: the host folds every
// Clifford into the frame D and hands each rotation its axis P = D sigma
// D^dag (FramePassDesc).  A rotation then splits every stored S that
// anticommutes with P into cos(t) S + i sin(t) P S (Table I's R rows
// conjugated by D), and i P S = +-(Pauli of key(S) ^ key(P)).  Duplicates
// are found through a hash index (key -> list position) instead of a sort:
// S and K = S ^ P anticommute with P together, so when both are present the
// pair is updated by the thread of the smaller key, and otherwise the child
// of S is appended.  Every weight is written by one thread from fixed
// inputs (the sum of two products, rounded as the sort-merge engine rounds
// it), so results do not depend on scheduling although the list order does.
__device__ __forceinline__ uint64_t frame_home(uint64_t key, int bits) {
    return (key * 0x9E3779B97F4A7C15ull) >> (64 - bits);
}

typedef unsigned long long FrameSlot __attribute__((ext_vector_type(2)));  // key, list position

__device__ __forceinline__ FrameSlot frame_slot(const FrameBuffers &f, uint64_t s) {
    return *reinterpret_cast<const FrameSlot *>(f.index + 2 * s);
}

// List position of `key`, or -1, given the slot `e` already read at probe
// position `s` (its home slot).  Slots only ever go from empty to a key, so
// an empty slot met on the probe path means the key was never inserted;
// keys this thread looks up are either older than the kernel or its own.
__device__ __forceinline__ long long frame_resolve(const FrameBuffers &f, uint64_t key, uint64_t s, FrameSlot e) {
    const uint64_t mask = (uint64_t)f.slots - 1;
    for (long long probe = 0; probe < f.slots; ++probe) {
        if (e.x == key) return (long long)e.y;
        if (e.x == kFrameEmpty) return -1;
        s = (s + 1) & mask;
        e = frame_slot(f, s);
    }
    return -1;
}

__device__ __forceinline__ long long frame_find(const FrameBuffers &f, uint64_t key) {
    const uint64_t s = frame_home(key, f.slot_bits);
    return frame_resolve(f, key, s, frame_slot(f, s));
}

__device__ __forceinline__ void frame_insert(const FrameBuffers &f, uint64_t key, uint64_t pos) {
    const uint64_t mask = (uint64_t)f.slots - 1;
    uint64_t s = frame_home(key, f.slot_bits);
    for (long long probe = 0; probe < f.slots; ++probe) {
        const unsigned long long prev = atomicCAS((unsigned long long *)(f.index + 2 * s),
                                                  (unsigned long long)kFrameEmpty, (unsigned long long)key);
        if (prev == kFrameEmpty || prev == key) {
            f.index[2 * s + 1] = pos;
            return;
        }
        s = (s + 1) & mask;
    }
}

// Sign of i P S as a multiple of the Hermitian Pauli of key(S) ^ key(P), for
// anticommuting Hermitian P (packed pmask, a = |x_P & z_P|) and S (packed
// key), with Y = iXZ: P S = i^(a + b + 2c - d) (Pauli of the XOR), where
// b = |x_S & z_S|, c = |z_P & x_S| (Z past X), d = |x' & z'| of the result.
__device__ __forceinline__ double frame_child_sign(uint64_t key, uint64_t pmask, int a, int n) {
    const uint64_t lo = (1ull << n) - 1ull;
    const uint64_t xs = key & lo, zs = key >> n, xp = pmask & lo, zp = pmask >> n;
    const int b = __popcll(xs & zs), c = __popcll(zp & xs), d = __popcll((xs ^ xp) & (zs ^ zp));
    return ((1 + a + b + 2 * c - d) & 3) == 0 ? 1.0 : -1.0;
}

// the merged weight of a pair: both products rounded to the storage type,
// summed in FP64 (the rounding points of the sort-merge engine)
template <typename T>
__device__ __forceinline__ double frame_merge2(double p, double q) {
    return (double)(T)p + (double)(T)q;
}

// Whole 16-byte slots (key empty, position 0) in one store each: writing
// only the key word would leave every cache line half written, which the
// memory side completes with a read.
__global__ void frame_clear_kernel(uint64_t *__restrict__ index, long long slots) {
    FrameSlot *sl = reinterpret_cast<FrameSlot *>(index);
    const FrameSlot empty = {kFrameEmpty, 0ull};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < slots; i += (long long)gridDim.x * blockDim.x)
        sl[i] = empty;
}

// The observable into the list and the index (one thread, in term order;
// repeated strings are summed).
template <typename T>
__global__ void frame_init_kernel(FrameBuffers f, const uint64_t *ox, const uint64_t *oz, const double *oc,
                                  int nterms) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    unsigned long long len = 0, over = 0;
    for (int t = 0; t < nterms; ++t) {
        const uint64_t key = (oz[t] << f.n) | ox[t];
        const long long j = frame_find(f, key);
        if (j >= 0) {
            stc<T>(f.coef, j, ldc<T>(f.coef, j) + oc[t]);
        } else if ((long long)len < f.cap) {
            f.keys[len] = key;
            stc<T>(f.coef, len, oc[t]);
            frame_insert(f, key, len);
            ++len;
        } else {
            over = 1;
        }
    }
    // the state "after pass -1": slot 2; pass 0 appends into slot 0
    f.cnt[2] = len;
    f.cnt[5] = 0;
    f.cnt[3] = 0;
    f.cnt[6] = over;
    *f.updates = 0;
}

// list length after pass `last` (-1: the observable)
__device__ __forceinline__ long long frame_len(const FrameBuffers &f, int last) {
    const int q = frame_slot_of(last);
    const long long t = (long long)(f.cnt[q] + f.cnt[3 + q]);
    return t < f.cap ? t : f.cap;
}

// One pass: its Clifford gates (already in the frame) and its rotation.
// Counters rotate over three slots, so no workgroup waits for another: the
// length entering pass `pass` is L + D of the previous slot (stable during
// this pass), this pass records it in its own slot and counts its children
// there, and clears the next slot for the pass after.
template <typename T>
__global__ __launch_bounds__(SP_BLOCK) void frame_pass_kernel(FrameBuffers f, FramePassDesc p,
                                                             const double *__restrict__ theta, int pass) {
#pragma clang fp contract(off)
    __shared__ int wsum[SP_BLOCK / 64];
    __shared__ unsigned long long tbase;
    const int q = frame_slot_of(pass), qprev = frame_slot_of(pass - 1), qnext = frame_slot_of(pass + 1);
    const long long T0 = frame_len(f, pass - 1);  // list length entering the pass
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *f.updates += (unsigned long long)T0 * (unsigned long long)p.ngates;
        f.cnt[q] = (unsigned long long)T0;
        f.cnt[3 + qnext] = 0;
        if (f.cnt[qprev] + f.cnt[3 + qprev] > (unsigned long long)f.cap) f.cnt[6] = 1;
    }
    const int n = f.n, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (p.rot_param < 0) return;
    double sn, cs;
    sincos(theta[p.rot_param], &sn, &cs);
    const double ssn = p.sign > 0 ? sn : -sn;
    const uint64_t lo = (1ull << n) - 1ull;
    const uint64_t xp = p.pmask & lo, zp = p.pmask >> n;
    const long long L = live_tiles(T0);
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        // all items' keys, then the first probe of every anticommuting item,
        // issued together: the lookups are random accesses, so they are
        // kept in flight side by side rather than one by one
        uint64_t key[SP_ITEMS], slot[SP_ITEMS], kc[SP_ITEMS];
        FrameSlot e[SP_ITEMS];
        double vc[SP_ITEMS], cw[SP_ITEMS];
        unsigned anti = 0, kids = 0;
#pragma unroll
        for (int it = 0; it < SP_ITEMS; ++it) {
            const long long i = t * SP_TILE + it * SP_BLOCK + threadIdx.x;
            key[it] = i < T0 ? f.keys[i] : 0;
            const bool a = i < T0 && ((__popcll((key[it] & lo) & zp) + __popcll((key[it] >> n) & xp)) & 1);
            anti |= (unsigned)a << it;
            slot[it] = frame_home(key[it] ^ p.pmask, f.slot_bits);
        }
        // the first probe and the weight of every anticommuting item, all
        // in flight before any is used
#pragma unroll
        for (int it = 0; it < SP_ITEMS; ++it)
            if ((anti >> it) & 1u) {
                e[it] = frame_slot(f, slot[it]);
                cw[it] = ldc<T>(f.coef, t * SP_TILE + it * SP_BLOCK + threadIdx.x);
            }
#pragma unroll
        for (int it = 0; it < SP_ITEMS; ++it) {
            kc[it] = 0;
            vc[it] = 0.0;
            if (!((anti >> it) & 1u)) continue;
            const long long i = t * SP_TILE + it * SP_BLOCK + threadIdx.x;
            const uint64_t K = key[it] ^ p.pmask;
            const long long j = frame_resolve(f, K, slot[it], e[it]);
            const double cS = cw[it];
            if (j < 0) {
                stc<T>(f.coef, i, cS * cs);
                kids |= 1u << it;
                kc[it] = K;
                vc[it] = cS * (frame_child_sign(key[it], p.pmask, p.a, n) * ssn);
            } else if (key[it] < K) {
                // both present: S's child lands on K and K's on S
                const double cK = ldc<T>(f.coef, j);
                const double gS = frame_child_sign(key[it], p.pmask, p.a, n) * ssn;
                const double gK = frame_child_sign(K, p.pmask, p.a, n) * ssn;
                stc<T>(f.coef, i, frame_merge2<T>(cS * cs, cK * gK));
                stc<T>(f.coef, j, frame_merge2<T>(cK * cs, cS * gS));
            }
        }
        // the tile's children: one counter update per tile, positions from
        // a workgroup scan of the per-thread counts
        const int mine = __popc(kids);
        int incl = mine;
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            int total = 0;
            for (int u = 0; u < SP_BLOCK / 64; ++u) total += wsum[u];
            tbase = total ? atomicAdd(f.cnt + 3 + q, (unsigned long long)total) : 0ull;
        }
        __syncthreads();
        int woff = 0;
        for (int u = 0; u < w; ++u) woff += wsum[u];
        unsigned long long pos = (unsigned long long)T0 + tbase + (unsigned long long)(woff + incl - mine);
#pragma unroll
        for (int it = 0; it < SP_ITEMS; ++it) {
            if (!((kids >> it) & 1u)) continue;
            if ((long long)pos < f.cap) {
                f.keys[pos] = kc[it];
                stc<T>(f.coef, (long long)pos, vc[it]);
                frame_insert(f, kc[it], pos);
            }
            ++pos;
        }
        __syncthreads();  // wsum and tbase are reused by the next tile
    }
}

// Strings whose actual form is made of I and Z only: the x part of the
// actual string is linear in the key (xrows), so the others are skipped at
// the cost of n parities; the kept ones replay every Clifford for their
// actual z and sign.
template <typename T>
__global__ __launch_bounds__(SP_BLOCK) void frame_x0_kernel(FrameBuffers f, const uint64_t *__restrict__ xrows,
                                                           const uint32_t *__restrict__ codes, int ncodes, int npasses,
                                                           uint64_t *__restrict__ ox, uint64_t *__restrict__ oz, void *oc,
                                                           long long *__restrict__ ocount) {
    __shared__ uint64_t rows[64];
    const int n = f.n, lane = threadIdx.x & 63;
    if (threadIdx.x < n) rows[threadIdx.x] = xrows[threadIdx.x];
    __syncthreads();
    const long long T0 = frame_len(f, npasses - 1);
    const int ql = frame_slot_of(npasses - 1);
    const uint64_t lo = (1ull << n) - 1ull;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        ocount[1] = (f.cnt[6] || f.cnt[ql] + f.cnt[3 + ql] > (unsigned long long)f.cap) ? 1 : 0;
    const long long L = live_tiles(T0);
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        for (int it = 0; it < SP_ITEMS; ++it) {
            const long long i = t * SP_TILE + it * SP_BLOCK + threadIdx.x;
            bool keep = false;
            uint64_t zz = 0;
            double v = 0.0;
            if (i < T0) {
                const uint64_t key = f.keys[i];
                unsigned odd = 0;
                for (int j = 0; j < n; ++j) odd |= (unsigned)__popcll(key & rows[j]) & 1u;
                if (!odd) {
                    uint64_t x = key & lo, z = key >> n;
                    unsigned neg = 0;
                    clifford_apply(x, z, neg, codes, 0, ncodes);
                    keep = true;
                    zz = z;
                    v = ldc<T>(f.coef, i);
                    if (neg) v = -v;
                }
            }
            const unsigned long long bal = __ballot(keep);
            if (bal) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd((unsigned long long *)ocount, (unsigned long long)__popcll(bal));
                base = __shfl(base, 0, 64);
                if (keep) {
                    const long long pos = (long long)(base + (unsigned long long)__popcll(bal & ((1ull << lane) - 1ull)));
                    ox[pos] = 0;
                    oz[pos] = zz;
                    stc<T>(oc, pos, v);
                }
            }
        }
    }
}

// Every string in its actual form, at its list position.
template <typename T>
__global__ __launch_bounds__(SP_BLOCK) void frame_materialize_kernel(FrameBuffers f, const uint32_t *__restrict__ codes,
                                                                    int ncodes, int npasses, uint64_t *__restrict__ ox,
                                                                    uint64_t *__restrict__ oz, void *oc,
                                                                    long long *__restrict__ ocount) {
    const long long T0 = frame_len(f, npasses - 1);
    const int ql = frame_slot_of(npasses - 1);
    const uint64_t lo = (1ull << f.n) - 1ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ocount[0] = T0;
        ocount[1] = (f.cnt[6] || f.cnt[ql] + f.cnt[3 + ql] > (unsigned long long)f.cap) ? 1 : 0;
    }
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < T0; i += (long long)gridDim.x * blockDim.x) {
        const uint64_t key = f.keys[i];
        uint64_t x = key & lo, z = key >> f.n;
        unsigned neg = 0;
        clifford_apply(x, z, neg, codes, 0, ncodes);
        ox[i] = x;
        oz[i] = z;
        const double v = ldc<T>(f.coef, i);
        stc<T>(oc, i, neg ? -v : v);
    }
}

// The ramp of a DENSE evaluation: the frame engine's strings (after its
// last pass), mapped through the frame's Clifford gates to their actual
// form, written into the 4^n weight array (already zero) at slot
// sum_q (x_q + 2 z_q) 4^q.  The list holds each string once, so plain
// stores suffice.
template <typename T>
__global__ __launch_bounds__(SP_BLOCK) void frame_to_dense_kernel(FrameBuffers f, const uint32_t *__restrict__ codes,
                                                                 int ncodes, int npasses, T *__restrict__ coef) {
    const long long T0 = frame_len(f, npasses - 1);
    const uint64_t lo = (1ull << f.n) - 1ull;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < T0; i += (long long)gridDim.x * blockDim.x) {
        const uint64_t key = f.keys[i];
        uint64_t x = key & lo, z = key >> f.n;
        unsigned neg = 0;
        clifford_apply(x, z, neg, codes, 0, ncodes);
        long long slot = 0;
        for (int q = 0; q < f.n; ++q) slot |= (long long)(((x >> q) & 1u) | (((z >> q) & 1u) << 1)) << (2 * q);
        const double v = ldc<T>(f.coef, i);
        coef[slot] = (T)(neg ? -v : v);
    }
}

__global__ void zero_ll_kernel(long long *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// ------------------------------------------------------------ launchers
// grid of a tile kernel: the capacity's tiles, at most SP_GRID workgroups
static int grid_for(const SparseBuffers &b) {
    const long long tiles = (b.cap2 + SP_TILE - 1) / SP_TILE;
    return (int)std::max<long long>(1, std::min<long long>(tiles, SP_GRID));
}

template <typename V>
static void launch_scan(V *a, const long long *count, int mult, SparseBuffers &b, long long *total, hipStream_t s,
                        int tile = SP_TILE) {
    hipLaunchKernelGGL(scan_reduce_kernel<V>, dim3(SCAN_BLOCKS), dim3(1024), 0, s, a, count, mult, tile, b.scan);
    hipLaunchKernelGGL(scan_apply_kernel<V>, dim3(SCAN_BLOCKS), dim3(1024), 0, s, a, count, mult, tile, b.scan,
                       total);
}

// Sort shapes (key bits per pass, terms per thread); entry 0 is the default.
struct SortShapeDef {
    int bits, items;
};
constexpr SortShapeDef kSortShapes[kSortShapeCount] = {{8, 8}, {8, 4}, {8, 16}, {7, 8}, {7, 16}, {6, 16}};
static int g_sort_shape[kSortClasses] = {0, 0, 0};

int sort_shape_class(long long cap2) { return cap2 <= (1ll << 18) ? 0 : (cap2 <= (1ll << 22) ? 1 : 2); }
void set_sort_shape(int cls, int shape) { g_sort_shape[cls] = shape; }
int sort_shape(int cls) { return g_sort_shape[cls]; }

long long sort_hist_entries(long long cap2) {
    long long most = 0;
    for (const SortShapeDef &d : kSortShapes) {
        const long long tile = (1ll << d.bits) * d.items;
        most = std::max(most, (1ll << d.bits) * ((cap2 + tile - 1) / tile));
    }
    return most;
}

// One LSD pass on key bits [shift, shift + BITS): histogram, scan, stable
// scatter into the second buffers, then the buffers swap.
template <int BITS, int ITEMS>
static void sort_pass(SparseBuffers &b, int n, int dtype_bytes, int shift, long long *total, hipStream_t s) {
    constexpr int BLOCK = 1 << BITS, TILE = BLOCK * ITEMS;
    const long long tiles = (b.cap2 + TILE - 1) / TILE;
    const int g = (int)std::max<long long>(1, std::min<long long>(tiles, SP_GRID));
    hipLaunchKernelGGL((sort_hist_kernel<BITS, ITEMS>), dim3(g), dim3(BLOCK), 0, s, b.x, b.z, b.count, n, shift,
                       b.hist);
    launch_scan<unsigned>(b.hist, b.count, BLOCK, b, total, s, TILE);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL((sort_scatter_kernel<double, BITS, ITEMS>), dim3(g), dim3(BLOCK), 0, s, b.x, b.z, b.c,
                           b.x2, b.z2, b.c2, b.count, n, shift, b.hist);
    else
        hipLaunchKernelGGL((sort_scatter_kernel<float, BITS, ITEMS>), dim3(g), dim3(BLOCK), 0, s, b.x, b.z, b.c,
                           b.x2, b.z2, b.c2, b.count, n, shift, b.hist);
    std::swap(b.x, b.x2);
    std::swap(b.z, b.z2);
    std::swap(b.c, b.c2);
}

template <int BITS, int ITEMS>
static void sort_all(SparseBuffers &b, int n, int dtype_bytes, long long *total, hipStream_t s) {
    for (int shift = 0; shift < 2 * n; shift += BITS) sort_pass<BITS, ITEMS>(b, n, dtype_bytes, shift, total, s);
}

hipError_t launch_sparse_init(SparseBuffers &b, int dtype_bytes, const uint64_t *x, const uint64_t *z,
                              const double *c, int nterms, hipStream_t s, double *dropped_total) {
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(sp_init_kernel<double>, dim3(1), dim3(64), 0, s, b.x, b.z, b.c, b.count, b.updates, x, z,
                           c, nterms, dropped_total);
    else
        hipLaunchKernelGGL(sp_init_kernel<float>, dim3(1), dim3(64), 0, s, b.x, b.z, b.c, b.count, b.updates, x, z, c,
                           nterms, dropped_total);
    return hipGetLastError();
}

hipError_t launch_sparse_pass(SparseBuffers &b, int dtype_bytes, const uint32_t *codes, const SparsePassDesc &p,
                              const double *theta, hipStream_t s, const SparseTrunc &tr) {
    const int g = grid_for(b);
    int *bc = b.tile_flags;
    long long *child_base = b.count + 2, *total = b.count + 4;
    const int mw = tr.on ? tr.max_weight : 64;
    double *drop = tr.on ? tr.dropped : nullptr;
    hipLaunchKernelGGL(pass_count_kernel, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.count, codes, p, bc, mw);
    launch_scan<int>(bc, b.count, 1, b, total, s);
    hipLaunchKernelGGL(pass_finalize_kernel, dim3(1), dim3(64), 0, s, b.count, total, b.cap2, b.updates, p.ngates,
                       child_base);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(pass_write_kernel<double>, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.c, child_base, b.cap2,
                           codes, p, theta, bc, mw, drop);
    else
        hipLaunchKernelGGL(pass_write_kernel<float>, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.c, child_base, b.cap2,
                           codes, p, theta, bc, mw, drop);
    if (drop)
        hipLaunchKernelGGL(trunc_total_kernel, dim3(1), dim3(SP_BLOCK), 0, s, drop, child_base,
                           (long long)b.max_tiles);
    return hipGetLastError();
}

hipError_t launch_sparse_merge(SparseBuffers &b, int n, int dtype_bytes, hipStream_t s, const SparseTrunc &tr) {
    const int g = grid_for(b);
    long long *old_count = b.count + 3, *total = b.count + 4;
    switch (g_sort_shape[sort_shape_class(b.cap2)]) {
    case 1: sort_all<8, 4>(b, n, dtype_bytes, total, s); break;
    case 2: sort_all<8, 16>(b, n, dtype_bytes, total, s); break;
    case 3: sort_all<7, 8>(b, n, dtype_bytes, total, s); break;
    case 4: sort_all<7, 16>(b, n, dtype_bytes, total, s); break;
    case 5: sort_all<6, 16>(b, n, dtype_bytes, total, s); break;
    default: sort_all<8, 8>(b, n, dtype_bytes, total, s); break;
    }
    int *bc = b.tile_flags;
    const int on = tr.on ? 1 : 0;
    const int mw = tr.on ? tr.max_weight : 64;
    const double eps = tr.on ? tr.eps : 0.0;
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(seg_count_kernel<double>, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.c, b.count, bc, on, mw,
                           eps);
    else
        hipLaunchKernelGGL(seg_count_kernel<float>, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.c, b.count, bc, on, mw,
                           eps);
    launch_scan<int>(bc, b.count, 1, b, total, s);
    hipLaunchKernelGGL(seg_finalize_kernel, dim3(1), dim3(64), 0, s, b.count, total, old_count);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(seg_write_kernel<double>, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.c, b.x2, b.z2, b.c2,
                           old_count, bc, on, mw, eps, tr.dropped);
    else
        hipLaunchKernelGGL(seg_write_kernel<float>, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.c, b.x2, b.z2, b.c2,
                           old_count, bc, on, mw, eps, tr.dropped);
    if (on)
        hipLaunchKernelGGL(trunc_total_kernel, dim3(1), dim3(SP_BLOCK), 0, s, tr.dropped, old_count,
                           (long long)b.max_tiles);
    std::swap(b.x, b.x2);
    std::swap(b.z, b.z2);
    std::swap(b.c, b.c2);
    return hipGetLastError();
}

hipError_t launch_sparse_readout(SparseBuffers &b, int dtype_bytes, double *partials, double *out, hipStream_t s) {
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(sp_readout_partial_kernel<double>, dim3(RO_BLOCKS), dim3(256), 0, s, b.x, b.c, b.count,
                           partials);
    else
        hipLaunchKernelGGL(sp_readout_partial_kernel<float>, dim3(RO_BLOCKS), dim3(256), 0, s, b.x, b.c, b.count,
                           partials);
    hipLaunchKernelGGL(sp_readout_final_kernel, dim3(1), dim3(64), 0, s, partials, b.count, out);
    return hipGetLastError();
}

static int frame_grid(const FrameBuffers &f) {
    const long long tiles = (f.cap + SP_TILE - 1) / SP_TILE;
    return (int)std::max<long long>(1, std::min<long long>(tiles, SP_GRID));
}

hipError_t launch_frame_init(FrameBuffers &f, int dtype_bytes, const uint64_t *x, const uint64_t *z, const double *c,
                             int nterms, hipStream_t s) {
    const long long blocks = std::min<long long>((f.slots + 255) / 256, 8192);
    hipLaunchKernelGGL(frame_clear_kernel, dim3((unsigned)blocks), dim3(256), 0, s, f.index, (long long)f.slots);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(frame_init_kernel<double>, dim3(1), dim3(64), 0, s, f, x, z, c, nterms);
    else
        hipLaunchKernelGGL(frame_init_kernel<float>, dim3(1), dim3(64), 0, s, f, x, z, c, nterms);
    return hipGetLastError();
}

hipError_t launch_frame_pass(FrameBuffers &f, int dtype_bytes, const FramePassDesc &p, const double *theta, int pass,
                             hipStream_t s) {
    // a pass without rotation only counts its gates: one workgroup
    const int g = p.rot_param >= 0 ? frame_grid(f) : 1;
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(frame_pass_kernel<double>, dim3(g), dim3(SP_BLOCK), 0, s, f, p, theta, pass);
    else
        hipLaunchKernelGGL(frame_pass_kernel<float>, dim3(g), dim3(SP_BLOCK), 0, s, f, p, theta, pass);
    return hipGetLastError();
}

hipError_t launch_frame_x0(FrameBuffers &f, int dtype_bytes, const uint64_t *xrows, const uint32_t *codes, int ncodes,
                           int npasses, SparseBuffers &out, hipStream_t s) {
    hipLaunchKernelGGL(zero_ll_kernel, dim3(1), dim3(64), 0, s, out.count, 8);
    const int g = frame_grid(f);
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(frame_x0_kernel<double>, dim3(g), dim3(SP_BLOCK), 0, s, f, xrows, codes, ncodes, npasses,
                           out.x, out.z, out.c, out.count);
    else
        hipLaunchKernelGGL(frame_x0_kernel<float>, dim3(g), dim3(SP_BLOCK), 0, s, f, xrows, codes, ncodes, npasses,
                           out.x, out.z, out.c, out.count);
    return hipGetLastError();
}

hipError_t launch_frame_to_dense(FrameBuffers &f, int dtype_bytes, const uint32_t *codes, int ncodes, int npasses,
                                 void *coef, hipStream_t s) {
    const int g = frame_grid(f) * SP_ITEMS;
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(frame_to_dense_kernel<double>, dim3(g), dim3(SP_BLOCK), 0, s, f, codes, ncodes, npasses,
                           (double *)coef);
    else
        hipLaunchKernelGGL(frame_to_dense_kernel<float>, dim3(g), dim3(SP_BLOCK), 0, s, f, codes, ncodes, npasses,
                           (float *)coef);
    return hipGetLastError();
}

hipError_t launch_frame_materialize(FrameBuffers &f, int dtype_bytes, const uint32_t *codes, int ncodes,
                                    int npasses, SparseBuffers &out, hipStream_t s) {
    hipLaunchKernelGGL(zero_ll_kernel, dim3(1), dim3(64), 0, s, out.count, 8);
    const int g = frame_grid(f) * SP_ITEMS;
    if (dtype_bytes == 8)
        hipLaunchKernelGGL(frame_materialize_kernel<double>, dim3(g), dim3(SP_BLOCK), 0, s, f, codes, ncodes, npasses,
                           out.x, out.z, out.c, out.count);
    else
        hipLaunchKernelGGL(frame_materialize_kernel<float>, dim3(g), dim3(SP_BLOCK), 0, s, f, codes, ncodes, npasses,
                           out.x, out.z, out.c, out.count);
    return hipGetLastError();
}

}  // namespace pp
