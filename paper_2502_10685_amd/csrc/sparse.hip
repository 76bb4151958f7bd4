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
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
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

// Exclusive scan, in place, of a[0, len) with len = mult * (live tiles of
// count[0]).  SCAN_BLOCKS workgroups each own one contiguous chunk: the first
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
                                                          int mult, long long *__restrict__ bsum) {
    __shared__ long long wsum[16];
    long long lo, hi;
    scan_chunk(mult * live_tiles(count[0]), lo, hi);
    long long s = 0;
    for (long long i = lo + threadIdx.x; i < hi; i += 1024) s += (long long)a[i];
    s = block_sum_1024(s, wsum);
    if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

template <typename V>
__global__ __launch_bounds__(1024) void scan_apply_kernel(V *__restrict__ a, const long long *__restrict__ count, int mult,
                                                         const long long *__restrict__ bsum, long long *__restrict__ total) {
    __shared__ long long wsum[16];
    __shared__ long long carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    long long lo, hi;
    scan_chunk(mult * live_tiles(count[0]), lo, hi);
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
__device__ __forceinline__ unsigned key_digit(uint64_t x, uint64_t z, int n, int s) {
    uint64_t v;
    if (s >= n) v = z >> (s - n);
    else if (s + RADIX_BITS <= n) v = x >> s;
    else v = (x >> s) | (z << (n - s));
    return (unsigned)(v & (RADIX - 1));
}

// Histograms are digit-major over the live tiles: hist[d * L + tile], so an
// exclusive scan of hist[0, RADIX * L) gives every (digit, tile) its output
// position.
__global__ __launch_bounds__(SP_BLOCK) void sort_hist_kernel(const uint64_t *__restrict__ x, const uint64_t *__restrict__ z,
                                                            const long long *__restrict__ count, int n, int shift,
                                                            unsigned *__restrict__ hist) {
    __shared__ unsigned h[RADIX];
    const long long T = count[0];
    const long long L = live_tiles(T);
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        for (int d = threadIdx.x; d < RADIX; d += SP_BLOCK) h[d] = 0;
        __syncthreads();
        const long long b0 = t * SP_TILE;
        for (int it = 0; it < SP_ITEMS; ++it) {
            const long long i = b0 + it * SP_BLOCK + threadIdx.x;
            if (i < T) atomicAdd(&h[key_digit(x[i], z[i], n, shift)], 1u);
        }
        __syncthreads();
        for (int d = threadIdx.x; d < RADIX; d += SP_BLOCK) hist[(long long)d * L + t] = h[d];
        __syncthreads();
    }
}

// Stable scatter of one tile.  Wave w owns the contiguous sub-tile
// [w*512, (w+1)*512) and walks it in chunks of 64; lanes with equal digits
// are matched with eight ballots, so the rank of a term is (terms of its
// digit in earlier waves) + (earlier chunks of its wave) + (lower lanes of
// its chunk).  Terms are staged in LDS in sorted order and written out so
// that each digit's run leaves the workgroup contiguously.
template <typename T>
__global__ __launch_bounds__(SP_BLOCK) void sort_scatter_kernel(const uint64_t *__restrict__ x, const uint64_t *__restrict__ z,
                                                               const void *c, uint64_t *__restrict__ xo,
                                                               uint64_t *__restrict__ zo, void *co,
                                                               const long long *__restrict__ count, int n, int shift,
                                                               const unsigned *__restrict__ hist) {
    __shared__ unsigned whist[SP_BLOCK / 64][RADIX];
    __shared__ unsigned tpre[RADIX];
    __shared__ unsigned goff[RADIX];
    __shared__ uint64_t sx[SP_TILE];
    __shared__ uint64_t sz[SP_TILE];
    __shared__ T sc[SP_TILE];
    const long long Tn = count[0];
    const long long L = live_tiles(Tn);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (long long t = blockIdx.x; t < L; t += gridDim.x) {
        const long long b0 = t * SP_TILE;
        for (int d = threadIdx.x; d < RADIX; d += SP_BLOCK) {
            for (int v = 0; v < SP_BLOCK / 64; ++v) whist[v][d] = 0;
            goff[d] = hist[(long long)d * L + t];
        }
        __syncthreads();

        uint64_t rx[SP_ITEMS], rz[SP_ITEMS];
        T rc[SP_ITEMS];
        unsigned rd[SP_ITEMS], rr[SP_ITEMS];
        for (int j = 0; j < SP_ITEMS; ++j) {
            const long long i = b0 + (long long)w * (SP_ITEMS * 64) + j * 64 + lane;
            const bool live = i < Tn;
            rx[j] = live ? x[i] : 0;
            rz[j] = live ? z[i] : 0;
            rc[j] = live ? ((const T *)c)[i] : (T)0;
            const unsigned d = key_digit(rx[j], rz[j], n, shift);
            unsigned long long peers = __ballot(live);
            for (int bt = 0; bt < RADIX_BITS; ++bt) {
                const unsigned long long bb = __ballot((d >> bt) & 1u);
                peers &= ((d >> bt) & 1u) ? bb : ~bb;
            }
            const unsigned before = whist[w][d];
            __builtin_amdgcn_wave_barrier();
            const int rank = __popcll(peers & lt);
            if (live && rank == 0) whist[w][d] = before + (unsigned)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            rd[j] = live ? d : RADIX;
            rr[j] = before + (unsigned)rank;
        }
        __syncthreads();
        // per digit: exclusive prefix over waves, then an exclusive scan of the
        // tile's digit totals (thread d owns digit d; SP_BLOCK == RADIX)
        {
            const int d = threadIdx.x;
            unsigned run = 0;
            for (int v = 0; v < SP_BLOCK / 64; ++v) {
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
        for (int j = 0; j < SP_ITEMS; ++j) {
            if (rd[j] < RADIX) {
                const unsigned pos = tpre[rd[j]] + whist[w][rd[j]] + rr[j];
                sx[pos] = rx[j];
                sz[pos] = rz[j];
                sc[pos] = rc[j];
            }
        }
        __syncthreads();
        const int valid = (int)((Tn - b0) < SP_TILE ? (Tn - b0) : SP_TILE);
        for (int i = threadIdx.x; i < valid; i += SP_BLOCK) {
            const unsigned d = key_digit(sx[i], sz[i], n, shift);
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

// ------------------------------------------------------------ launchers
// grid of a tile kernel: the capacity's tiles, at most SP_GRID workgroups
static int grid_for(const SparseBuffers &b) {
    const long long tiles = (b.cap2 + SP_TILE - 1) / SP_TILE;
    return (int)std::max<long long>(1, std::min<long long>(tiles, SP_GRID));
}

template <typename V>
static void launch_scan(V *a, const long long *count, int mult, SparseBuffers &b, long long *total, hipStream_t s) {
    hipLaunchKernelGGL(scan_reduce_kernel<V>, dim3(SCAN_BLOCKS), dim3(1024), 0, s, a, count, mult, b.scan);
    hipLaunchKernelGGL(scan_apply_kernel<V>, dim3(SCAN_BLOCKS), dim3(1024), 0, s, a, count, mult, b.scan, total);
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
    const int key_bits = 2 * n;
    long long *old_count = b.count + 3, *total = b.count + 4;
    for (int shift = 0; shift < key_bits; shift += RADIX_BITS) {
        hipLaunchKernelGGL(sort_hist_kernel, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.count, n, shift, b.hist);
        launch_scan<unsigned>(b.hist, b.count, RADIX, b, total, s);
        if (dtype_bytes == 8)
            hipLaunchKernelGGL(sort_scatter_kernel<double>, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.c, b.x2, b.z2,
                               b.c2, b.count, n, shift, b.hist);
        else
            hipLaunchKernelGGL(sort_scatter_kernel<float>, dim3(g), dim3(SP_BLOCK), 0, s, b.x, b.z, b.c, b.x2, b.z2,
                               b.c2, b.count, n, shift, b.hist);
        std::swap(b.x, b.x2);
        std::swap(b.z, b.z2);
        std::swap(b.c, b.c2);
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

}  // namespace pp
