// C ABI of libpauliprop (declared in include/pauliprop.h).
//
// A pp_circuit owns its gate list, angles, observable, the cached schedule
// (rebuilt only when the gates or a schedule option change, never for new
// angles) and its device buffers.  Every step of an evaluation runs in the
// kernels of dense.hip / sparse.hip; this file only plans, allocates and
// enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/pauliprop.h"
#include "plan.h"
#include "pp_device.h"

namespace {

thread_local std::string g_err;

pp_status fail(pp_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? PP_ERR_NOMEM : PP_ERR_DEVICE,         \
                        std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

// ------------------------------------------------------ device allocation
// Every device buffer of the library comes from the allocator installed with
// pp_set_allocator (for instance torch's caching allocator), or by default
// from the stream-ordered pool: hipMallocAsync on an internal stream, which
// is synchronized before the buffer is handed out, so the buffer can be used
// on any stream at once.  Each block remembers the hook that made it, so a
// later pp_set_allocator does not change where it is returned.  Before a
// block is returned the device is synchronized: enqueued work on any stream
// may still use it.
struct HookBlock {
    size_t bytes;
    pp_allocator hook;
    bool custom;
    int dev;
};
std::mutex g_alloc_mu;
pp_allocator g_hook{};
bool g_hook_set = false;
std::unordered_map<void *, HookBlock> g_blocks;
int64_t g_block_bytes = 0;
constexpr int kMaxDevices = 64;
hipStream_t g_pool_stream[kMaxDevices] = {};

hipError_t pool_stream(int dev, hipStream_t *s) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (!g_pool_stream[dev]) {
        hipError_t e = hipStreamCreateWithFlags(&g_pool_stream[dev], hipStreamNonBlocking);
        if (e != hipSuccess) {
            g_pool_stream[dev] = nullptr;
            return e;
        }
    }
    *s = g_pool_stream[dev];
    return hipSuccess;
}

hipError_t dev_alloc(void **p, size_t bytes) {
    *p = nullptr;
    bytes = std::max<size_t>(bytes, 1);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    pp_allocator hook;
    bool custom;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        hook = g_hook;
        custom = g_hook_set;
    }
    void *q = nullptr;
    if (custom) {
        q = hook.alloc(bytes, nullptr, hook.user);
        if (!q) return hipErrorOutOfMemory;
    } else {
        hipStream_t s = nullptr;
        if ((e = pool_stream(dev, &s)) != hipSuccess) return e;
        e = hipMallocAsync(&q, bytes, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            if (q) (void)hipFreeAsync(q, s);
            (void)hipGetLastError();
            return e;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_blocks[q] = HookBlock{bytes, hook, custom, dev};
        g_block_bytes += (int64_t)bytes;
    }
    *p = q;
    return hipSuccess;
}

void dev_free(void *p) {
    if (!p) return;
    HookBlock b;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        auto it = g_blocks.find(p);
        if (it == g_blocks.end()) return;
        b = it->second;
        g_blocks.erase(it);
        g_block_bytes -= (int64_t)b.bytes;
    }
    (void)hipDeviceSynchronize();
    if (b.custom) {
        b.hook.free(p, b.bytes, nullptr, b.hook.user);
    } else {
        hipStream_t s = nullptr;
        if (pool_stream(b.dev, &s) == hipSuccess) (void)hipFreeAsync(p, s);
    }
}

template <class T>
hipError_t dalloc(T **p, size_t count) {
    return dev_alloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
}

template <class T>
void dfree(T *&p) {
    dev_free((void *)p);
    p = nullptr;
}

__global__ void copy_f64_kernel(const double *src, double *dst, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = src[i];
}

__global__ void zero_u64_kernel(unsigned long long *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// Shifted parameter sets of the parameter-shift rule: set 2j has rotation j's
// angle raised by pi/2, set 2j+1 lowered by pi/2, every other rotation at its
// angle theta[rot_param[r]].
__global__ void psr_thetas_kernel(const double *__restrict__ theta, const int32_t *__restrict__ rot_param, int R,
                                  double *__restrict__ thetas) {
    const long long total = 2ll * R * R;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int set = (int)(i / R), r = (int)(i % R);
        double t = theta[rot_param[r]];
        if (r == set / 2) t += (set & 1) ? -M_PI_2 : M_PI_2;
        thetas[i] = t;
    }
}

// grad[p] = sum over the rotations r of parameter p, in gate order, of
// (f(theta_r + pi/2) - f(theta_r - pi/2)) / 2.
__global__ void psr_combine_kernel(const double *__restrict__ vals, const int32_t *__restrict__ off,
                                   const int32_t *__restrict__ rot, int nparams, double *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nparams) return;
    double g = 0.0;
    for (int i = off[p]; i < off[p + 1]; ++i) {
        const int r = rot[i];
        g += 0.5 * (vals[2 * r] - vals[2 * r + 1]);
    }
    grad[p] = g;
}

__global__ void compact_to_sparse_count_kernel(const unsigned long long *total, long long *count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        count[0] = (long long)*total;
        count[1] = 0;
    }
}

// ------------------------------------------- evaluation without allocation
// Working set of pp_evaluate_noalloc: a static device array (one per device,
// held until the process ends).  In host code `scratch` names a host-side
// stand-in, so its device address is resolved once per device with
// hipGetSymbolAddress and only that address is passed to kernels.
constexpr size_t kNoAllocBytes = (size_t)24 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kScratchDevices = 64;
unsigned char *g_scratch_dev[kScratchDevices] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (resolved once per
// device, with that device current: at the first pp_circuit_create there).
pp_status scratch_address(unsigned char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PP_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kScratchDevices) return fail(PP_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (unsigned char *)p;
    }
    *out = g_scratch_dev[dev];
    return PP_OK;
}


// Copies a circuit's device descriptors into the scratch array with their
// weight, map and result pointers redirected into it (no host copy: the
// launch sequence stays kernels only).
__global__ void noalloc_patch_kernel(const pp::ComposeDesc *comp_in, pp::ComposeDesc *comp_out,
                                     const pp::TilePassDesc *pass_in, pp::TilePassDesc *pass_out, int npass,
                                     const pp::ResidentDesc *res_in, pp::ResidentDesc *res_out, void *coef,
                                     double *maps, double *expval) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && comp_in) {
        pp::ComposeDesc d = *comp_in;
        d.maps = maps;
        *comp_out = d;
    }
    if (i == 0 && res_in) {
        pp::ResidentDesc d = *res_in;
        d.coef_in = nullptr;
        d.coef_out = nullptr;
        d.pres_out = nullptr;
        d.maps = maps;
        d.expval_out = expval;
        d.counters = nullptr;
        *res_out = d;
    }
    if (i < npass) {
        pp::TilePassDesc d = pass_in[i];
        d.coef = coef;
        d.pres = nullptr;
        d.maps = maps;
        d.counters = nullptr;
        pass_out[i] = d;
    }
}

constexpr int kResidentMaxN = 7;
constexpr int kDenseMaxN = 16;
constexpr int kDensityMaxN = 12;
// 32-bit tile offsets in the sparse kernels: 2x the capacity stays below 2^31
constexpr int64_t kSparseMaxTerms = (int64_t)1 << 29;
constexpr int kAutoDenseMaxN = 13;
constexpr int kLowQubits = 2;

// defaults measured by the autotuner on MI355X (batched probes, FP64)
int g_tile_qubits[17] = {0, 0, 0, 0, 0, 0, 0, 0, 6, 6, 6, 6, 6, 6, 6, 6, 6};
int default_tile_qubits(int n) { return n >= 8 && n <= 16 ? g_tile_qubits[n] : (n > 16 ? 6 : 5); }

// pinned staging for small asynchronous uploads, reused once the previous
// upload from it has completed
struct Staging {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    pp_status reserve(size_t bytes) {
        if (done) HIPCHK(hipEventSynchronize(done));
        if (bytes <= cap) return PP_OK;
        if (host) (void)hipHostFree(host);
        host = nullptr;
        cap = 0;
        HIPCHK(hipHostMalloc(&host, std::max<size_t>(bytes, 4096), hipHostMallocDefault));
        cap = std::max<size_t>(bytes, 4096);
        return PP_OK;
    }
    pp_status upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
        pp_status r = reserve(bytes);
        if (r != PP_OK) return r;
        std::memcpy(host, src, bytes);
        HIPCHK(hipMemcpyAsync(dst, host, bytes, hipMemcpyHostToDevice, s));
        if (!done) HIPCHK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        HIPCHK(hipEventRecord(done, s));
        return PP_OK;
    }
    void release() {
        if (done) (void)hipEventSynchronize(done);
        if (done) (void)hipEventDestroy(done);
        if (host) (void)hipHostFree(host);
        host = nullptr;
        done = nullptr;
        cap = 0;
    }
};

// ----------------------------------------------------------- kernel timing
enum ProfClass { PC_TILE = 0, PC_RES, PC_COMPOSE, PC_INIT, PC_READOUT, PC_SPASS, PC_SMERGE, PC_N };
const char *const kProfNames[PC_N] = {"tile_pass", "resident",  "compose",     "dense_init",
                                      "readout",   "sparse_pass", "sparse_merge"};

struct Prof {
    bool on = false;
    int capturing = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int cls; size_t start; int64_t launches; };
    std::vector<Rec> recs;  // class, index of the start event (stop: next), launches timed
    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            // timing only: no system-scope fence (no L2 write-back at each event)
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
};
Prof g_prof;

// Brackets the launches made during its lifetime with two recorded events.
// Each recorded event is a marker packet that delays the next kernel by a
// few microseconds, so runs of back-to-back tile passes are timed as a whole
// by TileSpan instead.
struct ProfScope {
    int cls;
    hipStream_t s;
    size_t idx = 0;
    bool active;
    ProfScope(int c, hipStream_t st) : cls(c), s(st) {
        active = g_prof.on && !g_prof.capturing;
        if (!active) return;
        idx = g_prof.used;
        hipEvent_t a = g_prof.take(), b = g_prof.take();
        active = a && b && hipEventRecord(a, s) == hipSuccess;
    }
    ~ProfScope() {
        if (!active) return;
        if (hipEventRecord(g_prof.pool[idx + 1], s) == hipSuccess) g_prof.recs.push_back({cls, idx, 1});
    }
};

// Times a run of consecutive tile-pass launches on one stream with one pair
// of events around the whole run (nothing else is launched on that stream in
// between); each launch is credited with the run's mean duration.  The passes
// then run back to back, and the mean equals the kernels' mean duration.
struct TileSpan {
    hipStream_t s = nullptr;
    size_t idx = 0;
    int64_t launches = 0;
    bool open = false;
    void begin(hipStream_t st) {
        if (open || !g_prof.on || g_prof.capturing) return;
        s = st;
        idx = g_prof.used;
        hipEvent_t a = g_prof.take(), b = g_prof.take();
        open = a && b && hipEventRecord(a, s) == hipSuccess;
        launches = 0;
    }
    void count() {
        if (open) ++launches;
    }
    void end() {
        if (!open) return;
        open = false;
        if (launches > 0 && hipEventRecord(g_prof.pool[idx + 1], s) == hipSuccess)
            g_prof.recs.push_back({PC_TILE, idx, launches});
    }
    ~TileSpan() { end(); }
};

}  // namespace

struct pp_circuit {
    int n = 0;
    pp_dtype dtype = PP_F64;
    pp_engine req = PP_ENGINE_AUTO;
    int engine = PP_ENGINE_DENSE;
    int dbytes = 8;

    pp::GateList g;
    bool have_gates = false;
    double *d_theta = nullptr;
    int theta_cap = 0;
    bool have_theta = false;
    std::vector<uint64_t> ox, oz;
    std::vector<double> oc;
    bool have_obs = false;
    uint64_t *d_ox = nullptr, *d_oz = nullptr;
    double *d_oc = nullptr;

    int track = 0, tile_opt = 0, use_graph = 0, block = 0;
    int64_t max_terms = 0;
    int keep_coef = 0;  // LDS-resident runs store their final weights (density matrix)
    // truncated propagation (SPARSE; off by default)
    double trunc_eps = 0.0;
    int trunc_w = 64;
    double *d_dropped = nullptr;  // per-tile dropped weights + the evaluation's total
    int fwd_maps = 0;   // maps are forward maps g P g^dag (the gate list is then read backwards)
    uint64_t gates_gen = 0;  // bumped by every pp_circuit_load_gates

    // density matrix: Heisenberg propagation of the inverse circuit
    pp_circuit *dm = nullptr;
    uint64_t dm_gen = ~0ull;
    // parameter-shift gradient: the same gates with one parameter per
    // rotation gate (rotation j reads parameter j), its shifted parameter
    // sets and results, and the rotations of each parameter in gate order
    pp_circuit *psr = nullptr;
    uint64_t psr_gen = ~0ull, psr_obs_gen = ~0ull;
    int32_t *d_psr_rot_param = nullptr;  // R: parameter of rotation j
    int32_t *d_psr_off = nullptr;        // n_params + 1: CSR offsets into d_psr_rot
    int32_t *d_psr_rot = nullptr;        // R: rotations grouped by parameter
    double *d_psr_thetas = nullptr;      // 2R x R shifted parameter sets
    double *d_psr_vals = nullptr;        // 2R results
    int32_t psr_R = 0;
    uint64_t obs_gen = 0;  // bumped by every pp_circuit_set_observable

    // schedule cache
    bool plan_valid = false;
    int plan_track = -1, plan_k = -1;
    void *plan_coef = nullptr;  // weight array the descriptors point at
    uint64_t plan_gen = 0;  // bumped whenever device descriptors change
    pp::DensePlan dplan;
    pp::SparsePlan splan;

    // dense buffers
    void *coef = nullptr;
    uint8_t *pres = nullptr;
    pp::DOp *d_ops = nullptr;
    double *d_maps = nullptr;
    int32_t *d_roff = nullptr, *d_rparam = nullptr;
    uint8_t *d_rop = nullptr;
    pp::TilePassDesc *d_pass = nullptr;
    pp::ResidentDesc *d_res = nullptr;
    pp::ComposeDesc *d_comp = nullptr;
    pp::ResidentDesc h_res{};
    pp::ComposeDesc h_comp{};
    std::vector<pp::TilePassDesc> h_pass;
    unsigned long long *d_counters = nullptr;
    double *d_result = nullptr;

    // sparse buffers
    pp::SparseBuffers sb{};
    void *sb_base[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // Clifford-frame engine (exact SPARSE runs with n <= 31): string list,
    // hash index, counters; its plan and the x rows of the final frame
    int frame_opt = 1;           // PP_OPT_SPARSE_FRAME
    int ramp_opt = 0;            // PP_OPT_FRAME_RAMP (DENSE)
    int plan_ramp_opt = 0;       // the ramp setting the plan was built with
    bool plan_seg = false;       // the plan has register segments (register-tile kernel selected)
    int64_t ramp_gate = -1;      // DENSE ramp: gates [ramp_gate, m) run in the Clifford frame
    pp::FrameBuffers fb{};
    pp::FramePlan fplan;
    uint64_t *d_xrows = nullptr;
    bool plan_frame = false;     // the plan's engine: frame (true) or sort-merge
    bool frame_ran = false;      // the last SPARSE evaluation used the frame
    bool frame_terms = false;    // sb holds the frame run's full final set
    uint32_t *d_codes = nullptr;
    double *d_partials = nullptr;

    // graph of one evaluation (tiled dense path)
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;

    // adjoint-gradient schedule and buffers (built on first pp_gradient)
    struct Grad {
        bool valid = false;
        int64_t every = -1;
        int k_heis = 0, k_fwd = 0;
        pp::GradPlan plan;
        pp::DOp *hops = nullptr, *fops = nullptr;
        double *hmaps = nullptr, *fmaps = nullptr;
        int32_t *hroff = nullptr, *hrparam = nullptr, *froff = nullptr, *frparam = nullptr;
        uint8_t *hrop = nullptr, *frop = nullptr;
        pp::ComposeDesc *comp = nullptr;  // [0] Heisenberg maps, [1] forward maps
        pp::TilePassDesc *hpass = nullptr;
        pp::ResidentDesc *hres = nullptr;  // one per segment (resident Heisenberg sweep)
        pp::GradPassDesc *gpass = nullptr;
        double *ckpt = nullptr, *rbuf = nullptr, *partials = nullptr, *rot_grad = nullptr;
        int32_t *slot_param = nullptr;
        int ncomp = 0;
        // graph of one gradient (PP_OPT_USE_GRAPH): results land in out
        // (<O>, then the gradient) and are copied to the caller's arrays
        hipGraph_t graph = nullptr;
        hipGraphExec_t gexec = nullptr;
        double *out = nullptr;
    } gr;

    // parameter sweep (pp_evaluate_thetas): per-set parameters, maps and
    // weights back to back, and the launch descriptors of the last sweep
    struct Sweep {
        int64_t cap = 0;  // parameter sets the buffers hold
        double *thetas = nullptr, *maps = nullptr;
        void *coef = nullptr;
        void *dbuf = nullptr;
        size_t dcap = 0;
        uint64_t gen = ~0ull;
        int64_t count = -1;
        double *out = nullptr;
        size_t comp_off = 0, res_off = 0, pass_off = 0;
        Staging staging;
    } sw;

    Staging staging;
    // recorded on the caller's stream after every theta upload, so that work
    // the library issues on streams of its own (the serving loop) is ordered
    // after the upload
    hipEvent_t theta_ev = nullptr;
    pp_stats st{};
    bool evaluated = false;
    int last_track = 0;
};

namespace {

void free_graph(pp_circuit *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
}

void free_grad(pp_circuit *c);

void free_sweep(pp_circuit *c) {
    c->sw.staging.release();
    dfree(c->sw.thetas);
    dfree(c->sw.maps);
    dfree(c->sw.coef);
    dfree(c->sw.dbuf);
    c->sw.cap = 0;
    c->sw.dcap = 0;
    c->sw.gen = ~0ull;
    c->sw.count = -1;
    c->sw.out = nullptr;
}

void free_plan_buffers(pp_circuit *c) {
    free_graph(c);
    free_grad(c);
    free_sweep(c);
    dfree(c->d_ops);
    dfree(c->d_maps);
    dfree(c->d_roff);
    dfree(c->d_rparam);
    dfree(c->d_rop);
    dfree(c->d_pass);
    dfree(c->d_res);
    dfree(c->d_comp);
    dfree(c->d_codes);
    dfree(c->d_xrows);
    c->plan_valid = false;
}

void free_grad_graph(pp_circuit *c) {
    auto &G = c->gr;
    if (G.gexec) (void)hipGraphExecDestroy(G.gexec);
    if (G.graph) (void)hipGraphDestroy(G.graph);
    G.gexec = nullptr;
    G.graph = nullptr;
    dfree(G.out);
}

void free_grad(pp_circuit *c) {
    auto &G = c->gr;
    free_grad_graph(c);
    if (!G.hops && !G.ckpt && !G.valid) return;
    dfree(G.hops); dfree(G.fops); dfree(G.hmaps); dfree(G.fmaps);
    dfree(G.hroff); dfree(G.hrparam); dfree(G.froff); dfree(G.frparam);
    dfree(G.hrop); dfree(G.frop); dfree(G.comp); dfree(G.hpass); dfree(G.hres); dfree(G.gpass);
    dfree(G.ckpt); dfree(G.rbuf); dfree(G.partials); dfree(G.rot_grad); dfree(G.slot_param);
    G.valid = false;
}

void free_state_buffers(pp_circuit *c) {
    free_graph(c);
    free_grad_graph(c);  // captured with this circuit's weight buffer
    dfree(c->coef);
    dfree(c->pres);
    dfree(c->d_counters);
    dfree(c->d_result);
    dfree(c->d_partials);
    for (void *&p : c->sb_base) dfree(p);
    dfree(c->sb.count);
    dfree(c->sb.scan);
    dfree(c->sb.updates);
    dfree(c->sb.hist);
    dfree(c->sb.tile_flags);
    dfree(c->d_dropped);
    c->sb = pp::SparseBuffers{};
    dfree(c->fb.keys);
    dev_free(c->fb.coef);
    dfree(c->fb.index);
    dfree(c->fb.cnt);
    dfree(c->fb.updates);
    c->fb = pp::FrameBuffers{};
}

int64_t dense_slots(int n) { return (int64_t)1 << (2 * n); }

std::atomic<uint64_t> g_plan_gen{0};

int tile_qubits_for(const pp_circuit *c) {
    if (c->n <= kResidentMaxN &&
        pp::resident_lds_bytes(c->n, c->dbytes, c->track != 0) + pp::kStaticLdsReserve <= (size_t)pp::max_lds_bytes())
        return c->n;
    int k = c->tile_opt > 0 ? c->tile_opt : default_tile_qubits(c->n);
    k = std::min(k, c->n - 1);
    k = std::max(k, kLowQubits + 2);
    k = std::min(k, 7);
    while (k > kLowQubits + 2 &&
           pp::resident_lds_bytes(k, c->dbytes, c->track != 0) + pp::kStaticLdsReserve > (size_t)pp::max_lds_bytes())
        --k;
    return k;
}

// weights = false: DENSE circuits get no 4^n weight array of their own (the
// serving loop runs them in buffers of its pool)
// The ramp of a DENSE evaluation (PP_OPT_FRAME_RAMP = t): the Heisenberg
// sweep starts in the Clifford frame, where the set holds only the strings
// it has, and hands over to the 4^n array once the set could exceed 4^n /
// 2^t strings.  A set of T strings entering a rotation leaves it with at
// most 2T (Table I: one child per anticommuting string) and Clifford gates
// keep its size, so `nterms * 2^(rotations so far)` bounds it; the frame
// runs the longest Heisenberg suffix of gates whose bound stays within the
// limit, which is also its capacity.
bool ramp_wanted(const pp_circuit *c) {
    return c->engine == PP_ENGINE_DENSE && c->ramp_opt > 0 && !c->track && c->n <= pp::kFrameMaxN;
}
int64_t ramp_limit(const pp_circuit *c) {
    return std::max<int64_t>((int64_t)1 << std::max(0, 2 * c->n - c->ramp_opt), 1);
}
// First gate of the frame suffix, or m when the ramp holds no gate.
int64_t ramp_switch_gate(const pp_circuit *c) {
    const int64_t limit = ramp_limit(c);
    int64_t bound = (int64_t)c->ox.size();
    if (bound > limit) return c->g.m;
    int64_t s = c->g.m;
    while (s > 0) {
        if (c->g.op[(size_t)s - 1] >= 3) {  // a rotation doubles the bound
            if (bound > limit / 2) break;
            bound *= 2;
        }
        --s;
    }
    return s;
}

pp_status ensure_state(pp_circuit *c, bool weights = true) {
    if (c->engine == PP_ENGINE_DENSE) {
        const int64_t slots = dense_slots(c->n);
        if (weights && !c->coef) {
            hipError_t e = dev_alloc(&c->coef, (size_t)slots * c->dbytes);
            if (e != hipSuccess) {
                c->coef = nullptr;
                return fail(PP_ERR_NOMEM, "dense weights: " + std::to_string(slots * c->dbytes) + " bytes");
            }
        }
        if (c->track && !c->pres) HIPCHK(dalloc(&c->pres, (size_t)slots));
    } else if (!c->sb.x) {
        int64_t cap = c->max_terms > 0 ? c->max_terms : (c->n <= 12 ? dense_slots(c->n) : ((int64_t)1 << 24));
        if (c->n <= 12) cap = std::min<int64_t>(cap, dense_slots(c->n));
        cap = std::max<int64_t>(cap, 1);
        const int64_t cap2 = 2 * cap;
        const int64_t tiles = (cap2 + 2047) / 2048;
        c->sb.cap2 = cap2;
        c->sb.max_tiles = tiles;
        for (int i = 0; i < 6; ++i) {
            const size_t bytes = (size_t)cap2 * ((i == 2 || i == 5) ? c->dbytes : 8);
            hipError_t e = dev_alloc(&c->sb_base[i], bytes);
            if (e != hipSuccess) {
                c->sb_base[i] = nullptr;
                return fail(PP_ERR_NOMEM, "sparse term buffers");
            }
        }
        c->sb.x = (uint64_t *)c->sb_base[0];
        c->sb.z = (uint64_t *)c->sb_base[1];
        c->sb.c = c->sb_base[2];
        c->sb.x2 = (uint64_t *)c->sb_base[3];
        c->sb.z2 = (uint64_t *)c->sb_base[4];
        c->sb.c2 = c->sb_base[5];
        HIPCHK(dalloc(&c->sb.count, 8));
        HIPCHK(dalloc(&c->sb.scan, 256));
        HIPCHK(dalloc(&c->sb.updates, 1));
        HIPCHK(dalloc(&c->sb.hist, (size_t)pp::sort_hist_entries(cap2)));
        HIPCHK(dalloc(&c->sb.tile_flags, (size_t)tiles));
        HIPCHK(dalloc(&c->d_dropped, (size_t)tiles + 1));
        HIPCHK(dalloc(&c->d_partials, 256));
    }
    const bool ramp = ramp_wanted(c);
    if (((c->engine == PP_ENGINE_SPARSE && c->n <= pp::kFrameMaxN && c->frame_opt) || ramp) && !c->fb.keys) {
        // index slots: a power of two of at least twice the list capacity
        const int64_t cap = ramp ? ramp_limit(c) : c->sb.cap2 / 2;
        int bits = 1;
        while (((int64_t)1 << bits) < 2 * cap) ++bits;
        pp::FrameBuffers f{};
        f.cap = cap;
        f.slots = (int64_t)1 << bits;
        f.slot_bits = bits;
        f.n = c->n;
        hipError_t e = dalloc(&f.keys, (size_t)cap);
        if (e == hipSuccess) e = dev_alloc(&f.coef, (size_t)cap * c->dbytes);
        if (e == hipSuccess) e = dalloc(&f.index, (size_t)(2 * f.slots));
        if (e == hipSuccess) e = dalloc(&f.cnt, 8);
        if (e == hipSuccess) e = dalloc(&f.updates, 1);
        if (e != hipSuccess) {
            dfree(f.keys);
            dev_free(f.coef);
            dfree(f.index);
            dfree(f.cnt);
            dfree(f.updates);
            return fail(PP_ERR_NOMEM, "Clifford-frame buffers");
        }
        c->fb = f;
    }
    if (!c->d_counters) HIPCHK(dalloc(&c->d_counters, 4));
    if (!c->d_result) HIPCHK(dalloc(&c->d_result, 1));
    return PP_OK;
}

template <class T>
pp_status upload_vec(T **dptr, const std::vector<T> &v) {
    dfree(*dptr);
    HIPCHK(dalloc(dptr, v.size()));
    if (!v.empty()) HIPCHK(hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return PP_OK;
}

// The Clifford-frame engine serves exact SPARSE evaluations with n <= 31;
// truncated runs and larger n take the sort-merge engine.
bool wants_frame(const pp_circuit *c) {
    return c->engine == PP_ENGINE_SPARSE && c->frame_opt && c->n <= pp::kFrameMaxN && c->trunc_eps == 0.0 &&
           c->trunc_w >= c->n && c->fb.keys;
}

pp_status ensure_plan(pp_circuit *c, bool weights = true) {
    pp_status r = ensure_state(c, weights);
    if (r != PP_OK) return r;
    const int k = c->engine == PP_ENGINE_DENSE ? tile_qubits_for(c) : 0;
    const bool frame = wants_frame(c);
    // 6-qubit tiles are ordered into register segments only for the
    // register-tile kernel; selecting it (or another kernel) re-plans
    const int tv6 = pp::tile_kernel_variant(6);
    const bool seg = c->engine == PP_ENGINE_DENSE && (tv6 == 3 || tv6 == 4);
    // the descriptors hold the weight pointer they were built with
    if (c->plan_valid && c->plan_track == c->track && c->plan_k == k && c->plan_coef == c->coef &&
        c->plan_frame == frame && c->plan_ramp_opt == c->ramp_opt && c->plan_seg == seg)
        return PP_OK;
    free_plan_buffers(c);
    if (c->track && c->engine == PP_ENGINE_DENSE && !c->pres) HIPCHK(dalloc(&c->pres, (size_t)dense_slots(c->n)));
    if (c->engine == PP_ENGINE_SPARSE) {
        c->splan = pp::plan_sparse(c->g);
        if ((r = upload_vec(&c->d_codes, c->splan.codes)) != PP_OK) return r;
        if (frame) {
            c->fplan = pp::plan_frame(c->g, c->splan);
            if ((r = upload_vec(&c->d_xrows, c->fplan.xrows)) != PP_OK) return r;
        }
    } else {
        c->ramp_gate = -1;
        if (ramp_wanted(c)) {
            const int64_t sw = ramp_switch_gate(c);
            if (sw < c->g.m) {
                // the frame runs gates [sw, m) (Heisenberg order: g_m first)
                pp::GateList suf;
                suf.n = c->g.n;
                suf.m = c->g.m - sw;
                suf.n_params = c->g.n_params;
                suf.op.assign(c->g.op.begin() + sw, c->g.op.end());
                suf.q0.assign(c->g.q0.begin() + sw, c->g.q0.end());
                suf.q1.assign(c->g.q1.begin() + sw, c->g.q1.end());
                suf.param.assign(c->g.param.begin() + sw, c->g.param.end());
                c->splan = pp::plan_sparse(suf);
                c->fplan = pp::plan_frame(suf, c->splan);
                if ((r = upload_vec(&c->d_codes, c->splan.codes)) != PP_OK) return r;
                c->ramp_gate = sw;
            }
        }
        if (c->ramp_gate >= 0) {
            pp::PlanOptions o;
            o.g_end = c->ramp_gate;  // the dense sweep takes the gates before the frame's
            o.segments = seg;
            c->dplan = pp::plan_dense_opts(c->g, k, kLowQubits, o);
        } else {
            pp::PlanOptions o;
            o.compose = o.group = o.reorder = c->track == 0;
            o.segments = seg;
            c->dplan = pp::plan_dense_opts(c->g, k, kLowQubits, o);
        }
        const pp::DensePlan &P = c->dplan;
        {
            // the kernels trust the schedule's digits and segment bounds
            const std::string bad = pp::plan_check(P, c->n);
            if (!bad.empty()) return fail(PP_ERR_STATE, "planner self-check: " + bad);
            if (!c->track && seg && !pp::plan_segmented(P))
                return fail(PP_ERR_STATE, "planner self-check: unsegmented pass");
        }
        if ((r = upload_vec(&c->d_ops, P.ops)) != PP_OK) return r;
        if ((r = upload_vec(&c->d_roff, P.roff)) != PP_OK) return r;
        if ((r = upload_vec(&c->d_rop, P.rop)) != PP_OK) return r;
        if ((r = upload_vec(&c->d_rparam, P.rparam)) != PP_OK) return r;
        HIPCHK(dalloc(&c->d_maps, (size_t)9 * std::max(P.nmaps(), 1)));
        c->h_comp = pp::ComposeDesc{c->d_roff, c->d_rop, c->d_rparam, c->d_theta, c->d_maps, P.nmaps(), c->fwd_maps};
        HIPCHK(dalloc(&c->d_comp, 1));
        HIPCHK(hipMemcpy(c->d_comp, &c->h_comp, sizeof(c->h_comp), hipMemcpyHostToDevice));
        if (P.resident) {
            pp::ResidentDesc &d = c->h_res;
            d = pp::ResidentDesc{};
            d.coef_out = (c->track || c->keep_coef) ? c->coef : nullptr;
            d.coef_in = c->ramp_gate >= 0 ? c->coef : nullptr;  // the ramp's strings
            d.pres_out = c->track ? c->pres : nullptr;
            d.ops = c->d_ops;
            d.maps = c->d_maps;
            d.obs_x = c->d_ox;
            d.obs_z = c->d_oz;
            d.obs_c = c->d_oc;
            d.expval_out = c->d_result;
            d.counters = c->d_counters;
            d.nops = (int32_t)P.ops.size();
            d.n = c->n;
            d.nterms = (int32_t)c->ox.size();
            HIPCHK(dalloc(&c->d_res, 1));
            HIPCHK(hipMemcpy(c->d_res, &d, sizeof(d), hipMemcpyHostToDevice));
        } else {
            c->h_pass.clear();
            const int ntiles = (int)((int64_t)1 << (2 * (c->n - k)));
            for (const pp::DensePass &ps : P.passes) {
                pp::TilePassDesc d{};
                d.coef = c->coef;
                d.pres = c->track ? c->pres : nullptr;
                d.ops = c->d_ops;
                d.maps = c->d_maps;
                d.counters = c->d_counters;
                d.n = c->n;
                d.k = k;
                d.op_begin = ps.op_begin;
                d.op_end = ps.op_end;
                d.tile_begin = 0;
                d.ntiles = ntiles;
                d.qubits = 0;
                for (int j = 0; j < k; ++j) d.qubits |= (uint64_t)ps.qubit[j] << (8 * j);
                d.reg_entry = pp::pass_reg_entry(P, ps);
                c->h_pass.push_back(d);
            }
            if ((r = upload_vec(&c->d_pass, c->h_pass)) != PP_OK) return r;
        }
    }
    c->plan_valid = true;
    c->plan_track = c->track;
    c->plan_k = k;
    c->plan_coef = c->coef;
    c->plan_frame = frame;
    c->plan_ramp_opt = c->ramp_opt;
    c->plan_seg = seg;
    c->plan_gen = ++g_plan_gen;
    return PP_OK;
}

pp_status check_ready(pp_circuit *c) {
    if (!c) return fail(PP_ERR_INVALID, "null circuit");
    if (!c->have_gates) return fail(PP_ERR_STATE, "gates not loaded");
    if (!c->have_theta) return fail(PP_ERR_STATE, "theta not set");
    if (!c->have_obs) return fail(PP_ERR_STATE, "observable not set");
    return PP_OK;
}

void fill_plan_stats(pp_circuit *c) {
    pp_stats &s = c->st;
    s.gates = c->g.m;
    s.engine = c->engine;
    if (c->engine == PP_ENGINE_DENSE) {
        const pp::DensePlan &P = c->dplan;
        s.ops = 0;
        for (const pp::DOp &d : P.ops) s.ops += d.kind != pp::DOP_GROUP && d.kind != pp::DOP_SEG;
        s.passes = (int64_t)P.passes.size() + (c->ramp_gate >= 0 ? (int64_t)c->fplan.passes.size() : 0);
        s.tile_qubits = P.k;
        const int64_t slots = dense_slots(c->n);
        const int64_t per = 2 * slots * (c->dbytes + (c->track ? 1 : 0));
        if (P.resident) {
            s.launches = 1 + (P.nmaps() > 0 ? 1 : 0);
            s.bytes_per_eval = 0;
        } else {
            s.launches = (int64_t)P.passes.size() + 3 + (P.nmaps() > 0 ? 1 : 0) + (c->track ? 1 : 0);
            s.bytes_per_eval = per * (int64_t)P.passes.size();
        }
    } else {
        const pp::SparsePlan &P = c->splan;
        s.ops = (int64_t)P.passes.size();
        s.passes = (int64_t)P.passes.size();
        s.tile_qubits = 0;
        int rot = 0;
        for (auto &p : P.passes) rot += p.rot_op >= 3;
        const int dig = (2 * c->n + 7) / 8;
        if (c->plan_frame)  // clear + init, one per pass, x0 + sort + readout
            s.launches = 2 + (int64_t)P.passes.size() + 2 + (3 * dig + 4) + 2;
        else
            s.launches = 2 + 3 * (int64_t)P.passes.size() + (int64_t)(rot + 1) * (3 * dig + 3) + 2;
        s.bytes_per_eval = 0;  // known after the run (48 or 40 bytes per update)
    }
}

pp_status enqueue_dense_body(pp_circuit *c, hipStream_t s, double *out) {
    const pp::DensePlan &P = c->dplan;
    if (c->track) hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, c->d_counters, 4);
    if (c->ramp_gate >= 0) {
        // the ramp: the gates after ramp_gate in the Clifford frame, then its
        // strings in their actual form into the zeroed 4^n array
        if ((int64_t)c->ox.size() > c->fb.cap) return fail(PP_ERR_CAPACITY, "observable larger than the ramp");
        HIPCHK(pp::launch_frame_init(c->fb, c->dbytes, c->d_ox, c->d_oz, c->d_oc, (int)c->ox.size(), s));
        const int np = (int)c->fplan.passes.size();
        for (int i = 0; i < np; ++i) {
            ProfScope ps(PC_SPASS, s);
            HIPCHK(pp::launch_frame_pass(c->fb, c->dbytes, c->fplan.passes[(size_t)i], c->d_theta, i, s));
        }
        ProfScope ps(PC_INIT, s);
        HIPCHK(pp::launch_dense_init(c->coef, nullptr, c->n, c->dbytes, c->d_ox, c->d_oz, c->d_oc, 0, s));
        HIPCHK(pp::launch_frame_to_dense(c->fb, c->dbytes, c->d_codes, (int)c->splan.codes.size(), np, c->coef, s));
    }
    if (P.nmaps() > 0) {
        ProfScope ps(PC_COMPOSE, s);
        HIPCHK(pp::launch_compose(c->d_comp, 1, s, P.nmaps()));
    }
    if (P.resident) {
        {
            ProfScope ps(PC_RES, s);
            HIPCHK(pp::launch_resident(c->d_res, 1, c->n, c->dbytes, c->track != 0, s));
        }
        hipLaunchKernelGGL(copy_f64_kernel, dim3(1), dim3(64), 0, s, c->d_result, out, 1);
        HIPCHK(hipGetLastError());
        return PP_OK;
    }
    if (c->ramp_gate < 0) {
        ProfScope ps(PC_INIT, s);
        HIPCHK(pp::launch_dense_init(c->coef, c->track ? c->pres : nullptr, c->n, c->dbytes, c->d_ox, c->d_oz,
                                     c->d_oc, (int)c->ox.size(), s));
    }
    const int shift = 2 * (c->n - P.k);
    TileSpan span;
    span.begin(s);
    for (size_t p = 0; p < P.passes.size(); ++p) {
        pp::TileGroups grp{};
        grp.ngroups = 1;
        grp.first_block[0] = 0;
        grp.first_block[1] = 1 << shift;
        grp.first_desc[0] = (int32_t)p;
        grp.shift[0] = shift;
        HIPCHK(pp::launch_tile_pass(c->d_pass, grp, P.k, c->dbytes, c->track != 0, s));
        span.count();
    }
    span.end();
    {
        ProfScope ps(PC_READOUT, s);
        HIPCHK(pp::launch_dense_readout(c->coef, c->n, c->dbytes, out, s));
    }
    if (c->track) HIPCHK(pp::launch_dense_count(c->pres, c->n, c->d_counters + 1, s));
    return PP_OK;
}

// Exact SPARSE evaluation in the Clifford frame: the observable into the
// list and index, one kernel per pass, then the strings whose actual form
// is made of I and Z sorted into canonical order and summed in that order.
pp_status enqueue_frame(pp_circuit *c, hipStream_t s, double *out) {
    if ((int64_t)c->ox.size() > c->fb.cap) return fail(PP_ERR_CAPACITY, "observable larger than the term capacity");
    HIPCHK(pp::launch_frame_init(c->fb, c->dbytes, c->d_ox, c->d_oz, c->d_oc, (int)c->ox.size(), s));
    const int np = (int)c->fplan.passes.size();
    for (int i = 0; i < np; ++i) {
        ProfScope ps(PC_SPASS, s);
        HIPCHK(pp::launch_frame_pass(c->fb, c->dbytes, c->fplan.passes[(size_t)i], c->d_theta, i, s));
    }
    {
        ProfScope ps(PC_SMERGE, s);
        HIPCHK(pp::launch_frame_x0(c->fb, c->dbytes, c->d_xrows, c->d_codes, (int)c->splan.codes.size(), np, c->sb,
                                   s));
        HIPCHK(pp::launch_sparse_merge(c->sb, c->n, c->dbytes, s));
    }
    {
        ProfScope ps(PC_READOUT, s);
        HIPCHK(pp::launch_sparse_readout(c->sb, c->dbytes, c->d_partials, out, s));
    }
    return PP_OK;
}

pp_status enqueue_sparse(pp_circuit *c, hipStream_t s, double *out) {
    if (c->plan_frame) return enqueue_frame(c, s, out);
    const pp::SparsePlan &P = c->splan;
    if ((int64_t)c->ox.size() > c->sb.cap2) return fail(PP_ERR_CAPACITY, "observable larger than the term capacity");
    pp::SparseTrunc tr;
    tr.on = (c->trunc_eps > 0.0 || c->trunc_w < c->n) ? 1 : 0;
    tr.max_weight = c->trunc_w;
    tr.eps = c->trunc_eps;
    tr.dropped = c->d_dropped;
    HIPCHK(pp::launch_sparse_init(c->sb, c->dbytes, c->d_ox, c->d_oz, c->d_oc, (int)c->ox.size(), s,
                                  c->d_dropped + c->sb.max_tiles));
    bool merged_last = true;
    for (const pp::SparsePassDesc &p : P.passes) {
        {
            ProfScope ps(PC_SPASS, s);
            HIPCHK(pp::launch_sparse_pass(c->sb, c->dbytes, c->d_codes, p, c->d_theta, s, tr));
        }
        merged_last = false;
        if (p.rot_op >= 3) {
            ProfScope ps(PC_SMERGE, s);
            HIPCHK(pp::launch_sparse_merge(c->sb, c->n, c->dbytes, s, tr));
            merged_last = true;
        }
    }
    if (!merged_last) {
        ProfScope ps(PC_SMERGE, s);
        HIPCHK(pp::launch_sparse_merge(c->sb, c->n, c->dbytes, s, tr));
    }
    {
        ProfScope ps(PC_READOUT, s);
        HIPCHK(pp::launch_sparse_readout(c->sb, c->dbytes, c->d_partials, out, s));
    }
    return PP_OK;
}

}  // namespace

// ===================================================================== API
extern "C" {

const char *pp_version(void) { return "pauliprop 0.1 (gfx950)"; }

const char *pp_last_error(void) { return g_err.c_str(); }

pp_status pp_set_allocator(const pp_allocator *a) {
    if (a && (!a->alloc || !a->free)) return fail(PP_ERR_INVALID, "allocator needs both alloc and free");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (a) {
        g_hook = *a;
        g_hook_set = true;
    } else {
        g_hook = pp_allocator{};
        g_hook_set = false;
    }
    return PP_OK;
}

pp_status pp_memory_in_use(int64_t *bytes, int64_t *blocks) {
    if (!bytes && !blocks) return fail(PP_ERR_INVALID, "null output");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (bytes) *bytes = g_block_bytes;
    if (blocks) *blocks = (int64_t)g_blocks.size();
    return PP_OK;
}

pp_status pp_circuit_create(int32_t n_qubits, pp_dtype dtype, pp_engine engine, pp_circuit **out) {
    if (!out) return fail(PP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 64) return fail(PP_ERR_INVALID, "n_qubits must be in [1, 64]");
    if (dtype != PP_F64 && dtype != PP_F32) return fail(PP_ERR_INVALID, "unknown dtype");
    if (engine != PP_ENGINE_AUTO && engine != PP_ENGINE_DENSE && engine != PP_ENGINE_SPARSE)
        return fail(PP_ERR_INVALID, "unknown engine");
    int resolved = engine;
    if (engine == PP_ENGINE_AUTO) resolved = n_qubits <= kAutoDenseMaxN ? PP_ENGINE_DENSE : PP_ENGINE_SPARSE;
    if (resolved == PP_ENGINE_DENSE && n_qubits > kDenseMaxN)
        return fail(PP_ERR_CAPACITY, "DENSE engine supports n <= 16");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PP_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    {
        // set-up of this device: the address of the static working array of
        // pp_evaluate_noalloc, resolved here so that the entry point itself
        // only reads it
        unsigned char *sp = nullptr;
        pp_status r = scratch_address(&sp);
        if (r != PP_OK) return r;
    }
    pp_circuit *c = new (std::nothrow) pp_circuit();
    if (!c) return fail(PP_ERR_NOMEM, "host allocation");
    c->n = n_qubits;
    c->dtype = dtype;
    c->dbytes = dtype == PP_F64 ? 8 : 4;
    c->req = engine;
    c->engine = resolved;
    c->g.n = n_qubits;
    *out = c;
    return PP_OK;
}

void pp_circuit_destroy(pp_circuit *c) {
    if (!c) return;
    // the streams of past evaluations may be gone (a server's, or the
    // caller's): wait for the whole device instead
    (void)hipDeviceSynchronize();
    if (c->dm) pp_circuit_destroy(c->dm);
    if (c->psr) pp_circuit_destroy(c->psr);
    dfree(c->d_psr_rot_param);
    dfree(c->d_psr_off);
    dfree(c->d_psr_rot);
    dfree(c->d_psr_thetas);
    dfree(c->d_psr_vals);
    free_plan_buffers(c);
    free_state_buffers(c);
    dfree(c->d_theta);
    dfree(c->d_ox);
    dfree(c->d_oz);
    dfree(c->d_oc);
    c->staging.release();
    if (c->theta_ev) (void)hipEventDestroy(c->theta_ev);
    delete c;
}

static pp_status validate_gates(int n, int64_t m, const uint8_t *op, const int32_t *q0, const int32_t *q1,
                                const int32_t *param, int32_t n_params) {
    if (m < 0 || n_params < 0) return fail(PP_ERR_INVALID, "negative size");
    if (m > 0 && (!op || !q0 || !q1 || !param)) return fail(PP_ERR_INVALID, "null gate array");
    for (int64_t g = 0; g < m; ++g) {
        if (op[g] > PP_RZ) return fail(PP_ERR_INVALID, "unknown op at gate " + std::to_string(g));
        if (q0[g] < 0 || q0[g] >= n) return fail(PP_ERR_INVALID, "qubit out of range at gate " + std::to_string(g));
        if (op[g] == PP_CX && (q1[g] < 0 || q1[g] >= n || q1[g] == q0[g]))
            return fail(PP_ERR_INVALID, "bad CX target at gate " + std::to_string(g));
        if (op[g] >= PP_RX && (param[g] < 0 || param[g] >= n_params))
            return fail(PP_ERR_INVALID, "parameter index out of range at gate " + std::to_string(g));
    }
    return PP_OK;
}

pp_status pp_plan_dense_info(int32_t n_qubits, int64_t m, const uint8_t *op, const int32_t *q0, const int32_t *q1,
                             const int32_t *param, int32_t n_params, int32_t k, int32_t compose, int32_t reorder,
                             int64_t *n_ops, int64_t *n_passes, int32_t *pass_ops, int64_t max_passes) {
    if (n_qubits < 1 || n_qubits > kDenseMaxN) return fail(PP_ERR_INVALID, "n_qubits must be in [1, 16]");
    if (k != n_qubits && (k < kLowQubits + 2 || k > 7 || k >= n_qubits))
        return fail(PP_ERR_INVALID, "k must be n or in [4, min(7, n-1)]");
    if (!n_ops || !n_passes || (max_passes > 0 && !pass_ops)) return fail(PP_ERR_INVALID, "null output");
    pp_status r = validate_gates(n_qubits, m, op, q0, q1, param, n_params);
    if (r != PP_OK) return r;
    pp::GateList g;
    g.n = n_qubits;
    g.m = m;
    g.op.assign(op, op + m);
    g.q0.assign(q0, q0 + m);
    g.q1.resize(m);
    g.param.resize(m);
    for (int64_t i = 0; i < m; ++i) {
        g.q1[i] = op[i] == PP_CX ? q1[i] : -1;
        g.param[i] = op[i] >= PP_RX ? param[i] : -1;
    }
    g.n_params = n_params;
    pp::DensePlan P = pp::plan_dense(g, k, kLowQubits, compose != 0, reorder != 0);
    const std::string bad = pp::plan_check(P, n_qubits);
    if (!bad.empty()) return fail(PP_ERR_STATE, "planner self-check: " + bad);
    if (compose && !pp::plan_segmented(P)) return fail(PP_ERR_STATE, "planner self-check: unsegmented pass");
    auto real_ops = [&](int b, int e) {
        int cnt = 0;
        for (int i = b; i < e; ++i) cnt += P.ops[i].kind != pp::DOP_GROUP && P.ops[i].kind != pp::DOP_SEG;
        return cnt;
    };
    *n_ops = real_ops(0, (int)P.ops.size());
    *n_passes = (int64_t)P.passes.size();
    for (int64_t i = 0; i < max_passes && i < (int64_t)P.passes.size(); ++i)
        pass_ops[i] = real_ops(P.passes[i].op_begin, P.passes[i].op_end);
    return PP_OK;
}

pp_status pp_plan_sparse_frame(int32_t n_qubits, int64_t m, const uint8_t *op, const int32_t *q0, const int32_t *q1,
                               const int32_t *param, int32_t n_params, int64_t max_passes, uint64_t *pmask,
                               int32_t *sign, int32_t *rot_param, int32_t *ngates, uint64_t *xrows,
                               int64_t *n_passes) {
    if (n_qubits < 1 || n_qubits > pp::kFrameMaxN) return fail(PP_ERR_INVALID, "n_qubits must be in [1, 31]");
    if (!n_passes || (max_passes > 0 && (!pmask || !sign || !rot_param || !ngates)))
        return fail(PP_ERR_INVALID, "null output");
    pp_status r = validate_gates(n_qubits, m, op, q0, q1, param, n_params);
    if (r != PP_OK) return r;
    pp::GateList g;
    g.n = n_qubits;
    g.m = m;
    g.op.assign(op, op + m);
    g.q0.assign(q0, q0 + m);
    g.q1.resize(m);
    g.param.resize(m);
    for (int64_t i = 0; i < m; ++i) {
        g.q1[i] = op[i] == PP_CX ? q1[i] : -1;
        g.param[i] = op[i] >= PP_RX ? param[i] : -1;
    }
    g.n_params = n_params;
    const pp::SparsePlan sp = pp::plan_sparse(g);
    const pp::FramePlan F = pp::plan_frame(g, sp);
    *n_passes = (int64_t)F.passes.size();
    for (int64_t i = 0; i < max_passes && i < (int64_t)F.passes.size(); ++i) {
        pmask[i] = F.passes[i].pmask;
        sign[i] = F.passes[i].sign;
        rot_param[i] = F.passes[i].rot_param;
        ngates[i] = F.passes[i].ngates;
    }
    if (xrows)
        for (int j = 0; j < n_qubits; ++j) xrows[j] = F.xrows[(size_t)j];
    return PP_OK;
}

pp_status pp_circuit_load_gates(pp_circuit *c, int64_t m, const uint8_t *op, const int32_t *q0, const int32_t *q1,
                                const int32_t *param, int32_t n_params) {
    if (!c) return fail(PP_ERR_INVALID, "null circuit");
    {
        pp_status r = validate_gates(c->n, m, op, q0, q1, param, n_params);
        if (r != PP_OK) return r;
    }
    if (c->engine == PP_ENGINE_DENSE && m > 0 && c->n > 32)
        return fail(PP_ERR_INVALID, "DENSE engine needs n <= 32");
    if ((int64_t)n_params > c->theta_cap) {
        double *nt = nullptr;
        HIPCHK(dalloc(&nt, (size_t)n_params));
        dfree(c->d_theta);
        c->d_theta = nt;
        c->theta_cap = n_params;
        c->have_theta = false;
    }
    if (n_params != c->g.n_params) c->have_theta = n_params == 0;
    c->g.m = m;
    c->g.op.assign(op, op + m);
    c->g.q0.assign(q0, q0 + m);
    c->g.q1.resize(m);
    c->g.param.resize(m);
    for (int64_t g = 0; g < m; ++g) {
        c->g.q1[g] = op[g] == PP_CX ? q1[g] : -1;
        c->g.param[g] = op[g] >= PP_RX ? param[g] : -1;
    }
    c->g.n_params = n_params;
    if (n_params == 0) c->have_theta = true;
    c->have_gates = true;
    c->gates_gen++;
    free_plan_buffers(c);
    c->evaluated = false;
    return PP_OK;
}

pp_status pp_circuit_set_theta(pp_circuit *c, const double *theta, int32_t on_device, void *stream) {
    if (!c) return fail(PP_ERR_INVALID, "null circuit");
    if (!c->have_gates) return fail(PP_ERR_STATE, "load gates first");
    const int np = c->g.n_params;
    if (np == 0) {
        c->have_theta = true;
        return PP_OK;
    }
    if (!theta) return fail(PP_ERR_INVALID, "theta is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (on_device) {
        HIPCHK(hipMemcpyAsync(c->d_theta, theta, sizeof(double) * np, hipMemcpyDeviceToDevice, s));
    } else {
        pp_status r = c->staging.upload(c->d_theta, theta, sizeof(double) * np, s);
        if (r != PP_OK) return r;
    }
    if (!c->theta_ev) HIPCHK(hipEventCreateWithFlags(&c->theta_ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(c->theta_ev, s));
    c->have_theta = true;
    return PP_OK;
}

pp_status pp_circuit_set_observable(pp_circuit *c, int64_t n_terms, const uint64_t *x, const uint64_t *z,
                                    const double *coeff) {
    if (!c) return fail(PP_ERR_INVALID, "null circuit");
    if (n_terms < 1 || n_terms > (1 << 30)) return fail(PP_ERR_INVALID, "n_terms must be in [1, 2^30]");
    if (!x || !z || !coeff) return fail(PP_ERR_INVALID, "null observable array");
    const uint64_t mask = c->n >= 64 ? ~0ull : ((1ull << c->n) - 1ull);
    for (int64_t k = 0; k < n_terms; ++k)
        if ((x[k] & ~mask) || (z[k] & ~mask)) return fail(PP_ERR_INVALID, "observable bit at or above n");
    uint64_t *dx = nullptr, *dz = nullptr;
    double *dc = nullptr;
    HIPCHK(dalloc(&dx, (size_t)n_terms));
    HIPCHK(dalloc(&dz, (size_t)n_terms));
    HIPCHK(dalloc(&dc, (size_t)n_terms));
    HIPCHK(hipMemcpy(dx, x, sizeof(uint64_t) * n_terms, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dz, z, sizeof(uint64_t) * n_terms, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dc, coeff, sizeof(double) * n_terms, hipMemcpyHostToDevice));
    dfree(c->d_ox);
    dfree(c->d_oz);
    dfree(c->d_oc);
    c->d_ox = dx;
    c->d_oz = dz;
    c->d_oc = dc;
    c->ox.assign(x, x + n_terms);
    c->oz.assign(z, z + n_terms);
    c->oc.assign(coeff, coeff + n_terms);
    c->have_obs = true;
    c->obs_gen++;
    free_plan_buffers(c);  // descriptors hold the observable pointers
    return PP_OK;
}

pp_status pp_circuit_set_option(pp_circuit *c, pp_option key, int64_t value) {
    if (!c) return fail(PP_ERR_INVALID, "null circuit");
    switch (key) {
    case PP_OPT_TRACK_TERMS:
        c->track = value ? 1 : 0;
        free_graph(c);
        return PP_OK;
    case PP_OPT_TILE_QUBITS:
        if (value != 0 && (value < 4 || value > 7)) return fail(PP_ERR_INVALID, "tile qubits must be 0 or 4..7");
        c->tile_opt = (int)value;
        free_graph(c);
        return PP_OK;
    case PP_OPT_MAX_TERMS:
        if (value < 0 || value > kSparseMaxTerms) return fail(PP_ERR_INVALID, "max terms must be 0..2^29");
        c->max_terms = value;
        free_state_buffers(c);
        free_plan_buffers(c);
        return PP_OK;
    case PP_OPT_USE_GRAPH:
        c->use_graph = value ? 1 : 0;
        free_graph(c);
        return PP_OK;
    case PP_OPT_BLOCK:
        if (value != 0 && (value < 64 || value > 1024 || (value & 63))) return fail(PP_ERR_INVALID, "bad block size");
        c->block = (int)value;
        return PP_OK;
    case PP_OPT_SPARSE_FRAME:
        c->frame_opt = value ? 1 : 0;
        free_graph(c);
        return PP_OK;
    case PP_OPT_FRAME_RAMP:
        if (value < 0 || value > 24) return fail(PP_ERR_INVALID, "frame ramp must be 0..24");
        if (c->engine == PP_ENGINE_DENSE && (int)value != c->ramp_opt) {
            free_plan_buffers(c);
            dfree(c->fb.keys);  // the ramp's capacity follows the setting
            dev_free(c->fb.coef);
            dfree(c->fb.index);
            dfree(c->fb.cnt);
            dfree(c->fb.updates);
            c->fb = pp::FrameBuffers{};
        }
        c->ramp_opt = (int)value;
        free_graph(c);
        return PP_OK;
    }
    return fail(PP_ERR_INVALID, "unknown option");
}

pp_status pp_evaluate(pp_circuit *c, void *stream, double *d_expval) {
    pp_status r = check_ready(c);
    if (r != PP_OK) return r;
    if (!d_expval) return fail(PP_ERR_INVALID, "d_expval is NULL");
    if ((r = ensure_plan(c)) != PP_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    fill_plan_stats(c);
    const bool sparse = c->engine == PP_ENGINE_SPARSE;
    if (c->use_graph && (sparse || !c->dplan.resident)) {
        // the whole evaluation is device-driven (no host synchronization),
        // so it is captured once and replayed; theta is read at replay
        if (!c->gexec) {
            hipStream_t cs;
            HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                g_prof.capturing++;
                r = sparse ? enqueue_sparse(c, cs, c->d_result) : enqueue_dense_body(c, cs, c->d_result);
                g_prof.capturing--;
                hipGraph_t gr = nullptr;
                hipError_t e2 = hipStreamEndCapture(cs, &gr);
                if (r == PP_OK && e2 == hipSuccess) {
                    c->graph = gr;
                    e2 = hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0);
                }
                if (e2 != hipSuccess && r == PP_OK) r = fail(PP_ERR_DEVICE, "graph capture failed");
            } else {
                r = fail(PP_ERR_DEVICE, "hipStreamBeginCapture failed");
            }
            (void)hipStreamDestroy(cs);
            if (r != PP_OK) {
                free_graph(c);
                return r;
            }
        }
        HIPCHK(hipGraphLaunch(c->gexec, s));
        hipLaunchKernelGGL(copy_f64_kernel, dim3(1), dim3(64), 0, s, c->d_result, d_expval, 1);
        HIPCHK(hipGetLastError());
    } else if (sparse) {
        r = enqueue_sparse(c, s, d_expval);
    } else {
        r = enqueue_dense_body(c, s, d_expval);
    }
    if (r != PP_OK) return r;
    c->evaluated = true;
    c->last_track = c->track;
    c->frame_ran = sparse && c->plan_frame;
    c->frame_terms = false;
    return PP_OK;
}

// pp_evaluate with the working set in the static scratch array: the
// circuit's device schedule (ops, recipes, descriptors) is read, its weights
// and maps are not touched; every launch takes the scratch address.
pp_status pp_evaluate_noalloc(pp_circuit *c, void *stream, double *d_expval) {
    pp_status r = check_ready(c);
    if (r != PP_OK) return r;
    if (!d_expval) return fail(PP_ERR_INVALID, "d_expval is NULL");
    if (c->engine != PP_ENGINE_DENSE || c->track || c->ramp_opt)
        return fail(PP_ERR_STATE, "pp_evaluate_noalloc runs DENSE circuits without term tracking or frame ramp");
    if (!c->plan_valid || c->plan_track != 0 || c->plan_k != tile_qubits_for(c))
        return fail(PP_ERR_STATE, "the circuit's schedule is not on the device: evaluate it once with "
                                  "pp_evaluate (or serve it) after its last change");
    const pp::DensePlan &P = c->dplan;
    unsigned char *base = nullptr;
    if ((r = scratch_address(&base)) != PP_OK) return r;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t npass = P.resident ? 0 : P.passes.size();
    const size_t off_comp = 0;
    const size_t off_res = up(sizeof(pp::ComposeDesc));
    const size_t off_pass = off_res + up(sizeof(pp::ResidentDesc));
    const size_t off_maps = off_pass + up(npass * sizeof(pp::TilePassDesc));
    const size_t off_coef = off_maps + up((size_t)9 * sizeof(double) * std::max(P.nmaps(), 1));
    const size_t coef_bytes = P.resident ? 0 : (size_t)dense_slots(c->n) * c->dbytes;
    if (off_coef + coef_bytes > kNoAllocBytes)
        return fail(PP_ERR_CAPACITY, "pp_evaluate_noalloc: working set of " + std::to_string(off_coef + coef_bytes) +
                                         " bytes exceeds the " + std::to_string(kNoAllocBytes) + "-byte array");
    hipStream_t s = (hipStream_t)stream;
    pp::ComposeDesc *comp = (pp::ComposeDesc *)(base + off_comp);
    pp::ResidentDesc *res = (pp::ResidentDesc *)(base + off_res);
    pp::TilePassDesc *pass = (pp::TilePassDesc *)(base + off_pass);
    double *maps = (double *)(base + off_maps);
    void *coef = base + off_coef;
    const int pblocks = (int)std::max<size_t>(1, (npass + 255) / 256);
    hipLaunchKernelGGL(noalloc_patch_kernel, dim3(pblocks), dim3(256), 0, s, c->d_comp, comp,
                       P.resident ? nullptr : c->d_pass, pass, (int)npass, P.resident ? c->d_res : nullptr, res, coef,
                       maps, d_expval);
    HIPCHK(hipGetLastError());
    if (P.nmaps() > 0) HIPCHK(pp::launch_compose(comp, 1, s, P.nmaps()));
    if (P.resident) {
        HIPCHK(pp::launch_resident(res, 1, c->n, c->dbytes, false, s));
        return PP_OK;
    }
    HIPCHK(pp::launch_dense_init(coef, nullptr, c->n, c->dbytes, c->d_ox, c->d_oz, c->d_oc, (int)c->ox.size(), s));
    const int shift = 2 * (c->n - P.k);
    for (size_t p = 0; p < npass; ++p) {
        pp::TileGroups grp{};
        grp.ngroups = 1;
        grp.first_block[0] = 0;
        grp.first_block[1] = 1 << shift;
        grp.first_desc[0] = (int32_t)p;
        grp.shift[0] = shift;
        HIPCHK(pp::launch_tile_pass(pass, grp, P.k, c->dbytes, false, s));
    }
    HIPCHK(pp::launch_dense_readout(coef, c->n, c->dbytes, d_expval, s));
    return PP_OK;
}

pp_status pp_get_stats(pp_circuit *c, pp_stats *out) {
    if (!c || !out) return fail(PP_ERR_INVALID, "null argument");
    if (c->evaluated) {
        HIPCHK(hipDeviceSynchronize());  // its stream may no longer exist
        if (c->engine == PP_ENGINE_SPARSE) {
            long long cnt[2] = {0, 0};
            unsigned long long upd = 0;
            if (c->frame_ran) {
                unsigned long long fc[7] = {0, 0, 0, 0, 0, 0, 0};
                HIPCHK(hipMemcpy(fc, c->fb.cnt, sizeof(fc), hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(&upd, c->fb.updates, sizeof(upd), hipMemcpyDeviceToHost));
                const int ql = pp::frame_slot_of((int)c->fplan.passes.size() - 1);
                const unsigned long long len = fc[ql] + fc[3 + ql];
                cnt[0] = (long long)std::min<unsigned long long>(len, (unsigned long long)c->fb.cap);
                cnt[1] = (fc[6] || len > (unsigned long long)c->fb.cap) ? 1 : 0;
            } else {
                HIPCHK(hipMemcpy(cnt, c->sb.count, sizeof(cnt), hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(&upd, c->sb.updates, sizeof(upd), hipMemcpyDeviceToHost));
            }
            c->st.term_updates = (int64_t)upd;
            c->st.final_terms = cnt[0];
            c->st.overflow = (int32_t)cnt[1];
            c->st.bytes_per_eval = (int64_t)upd * (16 + 2 * (int64_t)c->dbytes) ;
        } else if (c->last_track) {
            unsigned long long cnt[2] = {0, 0};
            HIPCHK(hipMemcpy(cnt, c->d_counters, sizeof(cnt), hipMemcpyDeviceToHost));
            c->st.term_updates = (int64_t)cnt[0];
            c->st.final_terms = (int64_t)cnt[1];
        }
    }
    *out = c->st;
    return PP_OK;
}

pp_status pp_get_terms(pp_circuit *c, void *stream, int64_t capacity, uint64_t *x, uint64_t *z, double *coeff,
                       int64_t *n_out) {
    if (!c || !n_out) return fail(PP_ERR_INVALID, "null argument");
    if (capacity > 0 && (!x || !z || !coeff)) return fail(PP_ERR_INVALID, "null output array");
    if (!c->evaluated) return fail(PP_ERR_STATE, "no evaluation yet");
    hipStream_t s = (hipStream_t)stream;
    if (c->engine == PP_ENGINE_DENSE && !c->last_track && c->dplan.resident)
        return fail(PP_ERR_STATE, "an untracked LDS-resident evaluation keeps its weights on chip: set "
                                  "PP_OPT_TRACK_TERMS = 1 for the evaluation");
    const uint64_t *sx = nullptr, *sz = nullptr;
    const void *sc = nullptr;
    int cbytes = c->dbytes;
    pp::SparseBuffers tmp{};
    void *tmp_base[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    long long count = 0;
    pp_status r = PP_OK;
    if (c->engine == PP_ENGINE_SPARSE) {
        if (c->frame_ran && !c->frame_terms) {
            // the actual strings of the frame run, sorted into canonical order
            HIPCHK(pp::launch_frame_materialize(c->fb, c->dbytes, c->d_codes, (int)c->splan.codes.size(),
                                                (int)c->fplan.passes.size(), c->sb, s));
            HIPCHK(pp::launch_sparse_merge(c->sb, c->n, c->dbytes, s));
            c->frame_terms = true;
        }
        HIPCHK(hipStreamSynchronize(s));
        long long cnt[2];
        HIPCHK(hipMemcpy(cnt, c->sb.count, sizeof(cnt), hipMemcpyDeviceToHost));
        if (cnt[1]) return fail(PP_ERR_CAPACITY, "term capacity was exceeded during the evaluation");
        count = cnt[0];
        sx = c->sb.x;
        sz = c->sb.z;
        sc = c->sb.c;
    } else {
        // compact present slots, then sort them into canonical order
        const int64_t slots = dense_slots(c->n);
        const int64_t tiles = (slots + 2047) / 2048;
        tmp.cap2 = slots;
        tmp.max_tiles = tiles;
        bool ok = true;
        for (int i = 0; i < 6 && ok; ++i) ok = dev_alloc(&tmp_base[i], (size_t)slots * 8) == hipSuccess;
        ok = ok && dalloc(&tmp.count, 8) == hipSuccess;
        ok = ok && dalloc(&tmp.scan, 256) == hipSuccess;
        ok = ok && dalloc(&tmp.updates, 1) == hipSuccess;
        ok = ok && dalloc(&tmp.hist, (size_t)pp::sort_hist_entries(slots)) == hipSuccess;
        ok = ok && dalloc(&tmp.tile_flags, (size_t)std::max<int64_t>(tiles, slots / 4096 + 1)) == hipSuccess;
        unsigned long long *total = c->d_counters + 2;
        if (ok) {
            tmp.x = (uint64_t *)tmp_base[0];
            tmp.z = (uint64_t *)tmp_base[1];
            tmp.c = tmp_base[2];
            tmp.x2 = (uint64_t *)tmp_base[3];
            tmp.z2 = (uint64_t *)tmp_base[4];
            tmp.c2 = tmp_base[5];
            hipError_t e = pp::launch_dense_compact(c->coef, c->last_track ? c->pres : nullptr, c->n, c->dbytes,
                                                    tmp.x, tmp.z, (double *)tmp.c,
                                                    total, tmp.tile_flags, nullptr, nullptr, s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(compact_to_sparse_count_kernel, dim3(1), dim3(64), 0, s, total, tmp.count);
                e = pp::launch_sparse_merge(tmp, c->n, 8, s);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) e = hipMemcpy(&count, tmp.count, sizeof(count), hipMemcpyDeviceToHost);
            if (e != hipSuccess) r = fail(PP_ERR_DEVICE, std::string("terms dump: ") + hipGetErrorString(e));
        } else {
            r = fail(PP_ERR_NOMEM, "terms dump scratch");
        }
        sx = tmp.x;
        sz = tmp.z;
        sc = tmp.c;
        cbytes = 8;
    }
    if (r == PP_OK) {
        *n_out = count;
        const int64_t k = std::min<int64_t>(count, capacity);
        if (k > 0) {
            hipError_t e = hipMemcpy(x, sx, sizeof(uint64_t) * k, hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(z, sz, sizeof(uint64_t) * k, hipMemcpyDeviceToHost);
            if (e == hipSuccess) {
                if (cbytes == 8) {
                    e = hipMemcpy(coeff, sc, sizeof(double) * k, hipMemcpyDeviceToHost);
                } else {
                    std::vector<float> f((size_t)k);
                    e = hipMemcpy(f.data(), sc, sizeof(float) * k, hipMemcpyDeviceToHost);
                    for (int64_t i = 0; i < k; ++i) coeff[i] = (double)f[i];
                }
            }
            if (e != hipSuccess) r = fail(PP_ERR_DEVICE, std::string("terms copy: ") + hipGetErrorString(e));
        }
        if (r == PP_OK && count > capacity) r = fail(PP_ERR_CAPACITY, "capacity smaller than the term count");
    }
    for (void *&p : tmp_base) dfree(p);
    dfree(tmp.count);
    dfree(tmp.scan);
    dfree(tmp.updates);
    dfree(tmp.hist);
    dfree(tmp.tile_flags);
    return r;
}

// Density matrix (the paper's toDM task).  rho = U |0><0| U^dag = 2^-n sum over
// the stabilizer group of U Z^z U^dag (eq. (3)): the 2^n strings Z^z with
// weight 1 are propagated in the Schrodinger picture, P -> g P g^dag, g_1
// first.  An internal circuit holds the gates in reverse order, so the dense
// engine (which processes its last gate first) meets g_1 first, and its maps
// are composed as forward maps (each gate's Heisenberg matrix transposed; CX
// is its own inverse).
pp_status pp_density_matrix(pp_circuit *c, void *stream, double *d_rho) {
    if (!c) return fail(PP_ERR_INVALID, "null circuit");
    if (!d_rho) return fail(PP_ERR_INVALID, "d_rho is NULL");
    if (c->n > kDensityMaxN) return fail(PP_ERR_INVALID, "density matrix needs n <= 12");
    if (!c->have_gates || !c->have_theta) return fail(PP_ERR_STATE, "load gates and theta first");
    hipStream_t s = (hipStream_t)stream;
    pp_status r = PP_OK;
    if (!c->dm || c->dm_gen != c->gates_gen) {
        if (c->dm) {
            pp_circuit_destroy(c->dm);
            c->dm = nullptr;
        }
        const int64_t m = c->g.m;
        std::vector<uint8_t> op((size_t)m);
        std::vector<int32_t> q0((size_t)m), q1((size_t)m), pa((size_t)m);
        for (int64_t i = 0; i < m; ++i) {
            const int64_t j = m - 1 - i;
            op[(size_t)i] = c->g.op[(size_t)j];
            q0[(size_t)i] = c->g.q0[(size_t)j];
            q1[(size_t)i] = c->g.q1[(size_t)j];
            pa[(size_t)i] = c->g.param[(size_t)j];
        }
        pp_circuit *a = nullptr;
        if ((r = pp_circuit_create(c->n, c->dtype, PP_ENGINE_DENSE, &a)) != PP_OK) return r;
        r = pp_circuit_load_gates(a, (int64_t)op.size(), op.data(), q0.data(), q1.data(), pa.data(), c->g.n_params);
        if (r == PP_OK) {
            const int64_t N = (int64_t)1 << c->n;
            std::vector<uint64_t> xs((size_t)N, 0), zs((size_t)N);
            std::vector<double> cs((size_t)N, 1.0);
            for (int64_t j = 0; j < N; ++j) zs[(size_t)j] = (uint64_t)j;
            r = pp_circuit_set_observable(a, N, xs.data(), zs.data(), cs.data());
        }
        if (r != PP_OK) {
            pp_circuit_destroy(a);
            return r;
        }
        a->keep_coef = 1;
        a->fwd_maps = 1;
        c->dm = a;
        c->dm_gen = c->gates_gen;
    }
    pp_circuit *a = c->dm;
    if (a->tile_opt != c->tile_opt && (r = pp_circuit_set_option(a, PP_OPT_TILE_QUBITS, c->tile_opt)) != PP_OK)
        return r;
    if ((r = pp_circuit_set_theta(a, c->d_theta, 1, stream)) != PP_OK) return r;
    if ((r = ensure_state(a)) != PP_OK) return r;
    if ((r = pp_evaluate(a, stream, a->d_result)) != PP_OK) return r;
    HIPCHK(pp::launch_density_decode(a->coef, a->n, a->dbytes, d_rho, s));
    return PP_OK;
}

pp_status pp_circuit_set_truncation(pp_circuit *c, double min_abs_coeff, int32_t max_weight) {
    if (!c) return fail(PP_ERR_INVALID, "null circuit");
    if (c->engine != PP_ENGINE_SPARSE) return fail(PP_ERR_STATE, "truncation needs the SPARSE engine");
    if (!(min_abs_coeff >= 0.0) || min_abs_coeff > 1e300) return fail(PP_ERR_INVALID, "min_abs_coeff must be >= 0");
    if (max_weight < 1 || max_weight > 64) return fail(PP_ERR_INVALID, "max_weight must be in [1, 64]");
    c->trunc_eps = min_abs_coeff;
    c->trunc_w = max_weight;
    free_graph(c);  // a captured evaluation holds the old cuts
    return PP_OK;
}

pp_status pp_get_truncation(pp_circuit *c, void *stream, double *dropped_abs) {
    if (!c || !dropped_abs) return fail(PP_ERR_INVALID, "null argument");
    if (c->engine != PP_ENGINE_SPARSE || !c->d_dropped || !c->evaluated)
        return fail(PP_ERR_STATE, "no SPARSE evaluation yet");
    if (c->frame_ran) {  // exact run: nothing dropped
        *dropped_abs = 0.0;
        return PP_OK;
    }
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    HIPCHK(hipMemcpy(dropped_abs, c->d_dropped + c->sb.max_tiles, sizeof(double), hipMemcpyDeviceToHost));
    return PP_OK;
}

}  // extern "C"

// ================================================================ batching
namespace {

// Device descriptors of the last batch, reused while the same circuits (with
// unchanged schedules) are evaluated into the same output array.
struct BatchCache {
    std::vector<const pp_circuit *> key;
    std::vector<uint64_t> gens;
    double *out = nullptr;
    void *dbuf = nullptr;
    size_t dcap = 0;
    Staging staging;
    hipEvent_t done = nullptr;
    // LDS-resident circuits run on a second stream, overlapping the tile passes
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    struct Launch { int kind; int group_n; int off; int nd; int nblocks; pp::TileGroups tg; };
    std::vector<Launch> launches;  // kind 0 compose, 1 resident, 2 tile pass
    int io_off = -1, io_max_n = 0;  // start/readout descriptors of the tiled circuits
    std::vector<int> tiled;        // indices of tiled circuits
    std::vector<int> single;       // indices evaluated one by one
    // the whole step captured once (every circuit sets PP_OPT_USE_GRAPH)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
};
BatchCache g_batch;

void free_batch_graph(BatchCache &B) {
    if (B.gexec) (void)hipGraphExecDestroy(B.gexec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    B.gexec = nullptr;
    B.graph = nullptr;
}

// The device work of one batch step on stream s: start weights, composed
// maps, LDS-resident circuits on the second stream, every tile pass, then
// the readouts.  It reads theta and writes the outputs through device
// pointers only, with no host synchronization, so it can be captured.
pp_status enqueue_batch_body(BatchCache &B, int dbytes, hipStream_t s) {
    unsigned char *base = (unsigned char *)B.dbuf;
    if (B.io_off >= 0) {
        ProfScope ps(PC_INIT, s);
        HIPCHK(pp::launch_dense_init_many((const pp::DenseIODesc *)(base + B.io_off), (int)B.tiled.size(),
                                          B.io_max_n, dbytes, s));
    }
    bool forked = false;
    TileSpan span;  // the tile passes come last in the list, all on s
    for (const auto &L : B.launches) {
        if (L.kind == 1 && !forked) {  // after the maps are composed
            HIPCHK(hipEventRecord(B.fork, s));
            HIPCHK(hipStreamWaitEvent(B.aux, B.fork, 0));
            forked = true;
        }
        if (L.kind == 2) {
            span.begin(s);
            HIPCHK(pp::launch_tile_pass((const pp::TilePassDesc *)(base + L.off), L.tg, L.group_n, dbytes, false, s));
            span.count();
            continue;
        }
        span.end();
        hipStream_t ls = L.kind == 1 ? B.aux : s;
        ProfScope ps(L.kind == 0 ? PC_COMPOSE : PC_RES, ls);
        if (L.kind == 0)
            HIPCHK(pp::launch_compose((const pp::ComposeDesc *)(base + L.off), L.nd, ls, L.nblocks));
        else
            HIPCHK(pp::launch_resident((const pp::ResidentDesc *)(base + L.off), L.nd, L.group_n, dbytes, false, ls));
    }
    span.end();
    if (forked) {
        HIPCHK(hipEventRecord(B.join, B.aux));
        HIPCHK(hipStreamWaitEvent(s, B.join, 0));
    }
    if (B.io_off >= 0) {
        ProfScope ps(PC_READOUT, s);
        HIPCHK(pp::launch_dense_readout_many((const pp::DenseIODesc *)(base + B.io_off), (int)B.tiled.size(), dbytes,
                                             s));
    }
    return PP_OK;
}

}  // namespace

extern "C" pp_status pp_evaluate_batch(pp_circuit *const *cs, int64_t count, void *stream, double *d_expvals) {
    if (count < 0 || (count > 0 && (!cs || !d_expvals))) return fail(PP_ERR_INVALID, "bad batch arguments");
    if (count == 0) return PP_OK;
    {
        // one circuit twice would scatter its observable into its one weight
        // array twice and put two workgroups on the same tiles
        std::unordered_set<const pp_circuit *> seen;
        seen.reserve((size_t)count);
        for (int64_t i = 0; i < count; ++i)
            if (cs[i] && !seen.insert(cs[i]).second)
                return fail(PP_ERR_INVALID, "circuit " + std::to_string(i) + " appears twice in the batch");
    }
    hipStream_t s = (hipStream_t)stream;
    pp_status r;
    int dbytes = -1;
    for (int64_t i = 0; i < count; ++i) {
        if ((r = check_ready(cs[i])) != PP_OK) return r;
        if ((r = ensure_plan(cs[i])) != PP_OK) return r;
        fill_plan_stats(cs[i]);
        if (cs[i]->engine == PP_ENGINE_DENSE && !cs[i]->track) {
            if (dbytes >= 0 && dbytes != cs[i]->dbytes) return fail(PP_ERR_INVALID, "mixed dtypes in one batch");
            dbytes = cs[i]->dbytes;
        }
    }
    BatchCache &B = g_batch;
    bool hit = B.out == d_expvals && B.key.size() == (size_t)count;
    for (int64_t i = 0; hit && i < count; ++i) hit = B.key[i] == cs[i] && B.gens[i] == cs[i]->plan_gen;
    if (!hit) {
        if (B.done) HIPCHK(hipEventSynchronize(B.done));
        free_batch_graph(B);  // it holds the old descriptors
        B.key.assign(cs, cs + count);
        B.gens.resize(count);
        for (int64_t i = 0; i < count; ++i) B.gens[i] = cs[i]->plan_gen;
        B.out = d_expvals;
        B.launches.clear();
        B.tiled.clear();
        B.single.clear();
        std::vector<unsigned char> blob;
        auto append = [&](const void *p, size_t bytes) {
            const size_t off = blob.size();
            blob.resize(off + ((bytes + 15) & ~size_t(15)));
            std::memcpy(blob.data() + off, p, bytes);
            return (int)off;
        };
        std::vector<pp::ComposeDesc> comp;
        int comp_max = 1;
        std::vector<std::vector<int>> res_by_n(kResidentMaxN + 1);
        for (int64_t i = 0; i < count; ++i) {
            pp_circuit *c = cs[i];
            if (c->engine != PP_ENGINE_DENSE || c->track || c->ramp_gate >= 0) {  // evaluated one by one
                B.single.push_back((int)i);
                continue;
            }
            if (c->dplan.nmaps() > 0) comp.push_back(c->h_comp);
            comp_max = std::max(comp_max, c->dplan.nmaps());
            if (c->dplan.resident) res_by_n[c->n].push_back((int)i);
            else B.tiled.push_back((int)i);
        }
        if (!comp.empty())
            B.launches.push_back({0, 0, append(comp.data(), comp.size() * sizeof(comp[0])), (int)comp.size(), comp_max, {}});
        B.io_off = -1;
        B.io_max_n = 0;
        if (!B.tiled.empty()) {
            std::vector<pp::DenseIODesc> io;
            for (int i : B.tiled) {
                pp_circuit *c = cs[i];
                io.push_back(pp::DenseIODesc{c->coef, c->d_ox, c->d_oz, c->d_oc, d_expvals + i, c->n,
                                             (int32_t)c->ox.size()});
                B.io_max_n = std::max(B.io_max_n, c->n);
            }
            B.io_off = append(io.data(), io.size() * sizeof(io[0]));
        }
        // resident groups, largest size class first, longest circuits first
        for (int n = kResidentMaxN; n >= 1; --n) {
            auto &v = res_by_n[n];
            if (v.empty()) continue;
            std::stable_sort(v.begin(), v.end(),
                             [&](int a, int b) { return cs[a]->dplan.ops.size() > cs[b]->dplan.ops.size(); });
            std::vector<pp::ResidentDesc> rd;
            for (int i : v) {
                pp::ResidentDesc d = cs[i]->h_res;
                d.expval_out = d_expvals + i;
                rd.push_back(d);
            }
            B.launches.push_back({1, n, append(rd.data(), rd.size() * sizeof(rd[0])), (int)rd.size(), 0, {}});
        }
        // tiled circuits: pass l of every circuit that has one, per tile size;
        // within a launch, descriptors are grouped by tile count
        for (int k = 4; k <= 7; ++k) {
            std::vector<int> grp;
            size_t maxp = 0;
            for (int i : B.tiled)
                if (cs[i]->dplan.k == k) {
                    grp.push_back(i);
                    maxp = std::max(maxp, cs[i]->dplan.passes.size());
                }
            std::stable_sort(grp.begin(), grp.end(), [&](int a, int b) { return cs[a]->n > cs[b]->n; });
            for (size_t l = 0; l < maxp; ++l) {
                // within one n, circuits whose pass l holds more ops come
                // first: workgroups take tiles with a fixed stride, so the
                // last round of tiles is the light one
                std::vector<int> order;
                for (int i : grp)
                    if (l < cs[i]->h_pass.size()) order.push_back(i);
                std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                    if (cs[a]->n != cs[b]->n) return cs[a]->n > cs[b]->n;
                    const pp::TilePassDesc &pa = cs[a]->h_pass[l], &pb = cs[b]->h_pass[l];
                    return pa.op_end - pa.op_begin > pb.op_end - pb.op_begin;
                });
                std::vector<pp::TilePassDesc> td;
                pp::TileGroups tg{};
                int run = 0, last_n = -1;
                for (int i : order) {
                    pp::TilePassDesc d = cs[i]->h_pass[l];
                    if (d.n != last_n) {
                        if (tg.ngroups == pp::kMaxTileGroups) {
                            tg.first_block[tg.ngroups] = run;
                            B.launches.push_back({2, k, append(td.data(), td.size() * sizeof(td[0])), (int)td.size(),
                                                  run, tg});
                            td.clear();
                            tg = pp::TileGroups{};
                            run = 0;
                        }
                        tg.first_block[tg.ngroups] = run;
                        tg.first_desc[tg.ngroups] = (int32_t)td.size();
                        tg.shift[tg.ngroups] = 2 * (d.n - k);
                        tg.ngroups++;
                        last_n = d.n;
                    }
                    d.tile_begin = run;
                    run += d.ntiles;
                    td.push_back(d);
                }
                tg.first_block[tg.ngroups] = run;
                B.launches.push_back({2, k, append(td.data(), td.size() * sizeof(td[0])), (int)td.size(), run, tg});
            }
        }
        if (blob.size() > B.dcap) {
            if (B.dbuf) HIPCHK(hipStreamSynchronize(s));
            dfree(B.dbuf);
            B.dcap = 0;
            HIPCHK(dev_alloc(&B.dbuf, blob.size()));
            B.dcap = blob.size();
        }
        if (!blob.empty()) {
            r = B.staging.upload(B.dbuf, blob.data(), blob.size(), s);
            if (r != PP_OK) return r;
        }
    }
    bool any_res = false;
    for (const auto &L : B.launches) any_res = any_res || L.kind == 1;
    if (any_res && !B.aux) {
        HIPCHK(hipStreamCreateWithFlags(&B.aux, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&B.fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&B.join, hipEventDisableTiming));
    }
    bool graph = B.single.empty();
    for (int64_t i = 0; graph && i < count; ++i) graph = cs[i]->use_graph != 0;
    if (graph) {
        if (!B.gexec) {
            hipStream_t cap;
            HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                g_prof.capturing++;
                r = enqueue_batch_body(B, dbytes, cap);
                g_prof.capturing--;
                hipGraph_t gr = nullptr;
                hipError_t e2 = hipStreamEndCapture(cap, &gr);
                if (r == PP_OK && e2 == hipSuccess) {
                    B.graph = gr;
                    e2 = hipGraphInstantiate(&B.gexec, gr, nullptr, nullptr, 0);
                } else if (gr) {
                    (void)hipGraphDestroy(gr);
                }
                if (e2 != hipSuccess && r == PP_OK) r = fail(PP_ERR_DEVICE, "batch graph capture failed");
            } else {
                r = fail(PP_ERR_DEVICE, "hipStreamBeginCapture failed");
            }
            (void)hipStreamDestroy(cap);
            if (r != PP_OK) {
                free_batch_graph(B);
                return r;
            }
        }
        HIPCHK(hipGraphLaunch(B.gexec, s));
    } else if ((r = enqueue_batch_body(B, dbytes, s)) != PP_OK) {
        return r;
    }
    for (int i : B.single)
        if ((r = pp_evaluate(cs[i], stream, d_expvals + i)) != PP_OK) return r;
    if (!B.done) HIPCHK(hipEventCreateWithFlags(&B.done, hipEventDisableTiming));
    HIPCHK(hipEventRecord(B.done, s));
    for (int64_t i = 0; i < count; ++i) {
        cs[i]->evaluated = true;
        cs[i]->last_track = cs[i]->track;
    }
    return PP_OK;
}

namespace {

pp_status ensure_grad(pp_circuit *c, int64_t every) {
    auto &G = c->gr;
    if (G.valid && G.every == every) return PP_OK;
    free_grad(c);
    const int n = c->n;
    const int k_heis = tile_qubits_for(c);
    const int k_fwd = n <= 6 ? n : 6;
    G.plan = pp::plan_gradient(c->g, k_heis, k_fwd, kLowQubits, every);
    const pp::GradPlan &P = G.plan;
    for (const pp::DensePlan *part : {&P.heis, &P.fwd}) {
        const std::string bad = pp::plan_check(*part, n);
        if (!bad.empty()) return fail(PP_ERR_STATE, "planner self-check: " + bad);
    }
    if (!pp::plan_segmented(P.heis)) return fail(PP_ERR_STATE, "planner self-check: unsegmented pass");
    pp_status r;
    if ((r = upload_vec(&G.hops, P.heis.ops)) != PP_OK) return r;
    if ((r = upload_vec(&G.hroff, P.heis.roff)) != PP_OK) return r;
    if ((r = upload_vec(&G.hrop, P.heis.rop)) != PP_OK) return r;
    if ((r = upload_vec(&G.hrparam, P.heis.rparam)) != PP_OK) return r;
    if ((r = upload_vec(&G.fops, P.fwd.ops)) != PP_OK) return r;
    if ((r = upload_vec(&G.froff, P.fwd.roff)) != PP_OK) return r;
    if ((r = upload_vec(&G.frop, P.fwd.rop)) != PP_OK) return r;
    if ((r = upload_vec(&G.frparam, P.fwd.rparam)) != PP_OK) return r;
    if ((r = upload_vec(&G.slot_param, P.slot_param)) != PP_OK) return r;
    HIPCHK(dalloc(&G.hmaps, (size_t)9 * std::max(P.heis.nmaps(), 1)));
    HIPCHK(dalloc(&G.fmaps, (size_t)9 * std::max(P.fwd.nmaps(), 1)));
    std::vector<pp::ComposeDesc> comp;
    if (P.heis.nmaps() > 0) comp.push_back({G.hroff, G.hrop, G.hrparam, c->d_theta, G.hmaps, P.heis.nmaps(), 0});
    if (P.fwd.nmaps() > 0) comp.push_back({G.froff, G.frop, G.frparam, c->d_theta, G.fmaps, P.fwd.nmaps(), 0});
    G.ncomp = (int)comp.size();
    if ((r = upload_vec(&G.comp, comp)) != PP_OK) return r;
    const size_t S = P.bounds.size() - 1;
    const int64_t slots = dense_slots(n);
    if (P.heis.resident) {
        std::vector<pp::ResidentDesc> rd;
        for (size_t sg = 0; sg < S; ++sg) {
            const pp::DensePass &ps = P.heis.passes[P.heis_pass_begin[sg]];
            pp::ResidentDesc d{};
            d.coef_in = sg + 1 == S ? nullptr : c->coef;
            d.coef_out = c->coef;
            d.ops = G.hops + ps.op_begin;
            d.maps = G.hmaps;
            d.obs_x = c->d_ox;
            d.obs_z = c->d_oz;
            d.obs_c = c->d_oc;
            d.expval_out = c->d_result;
            d.counters = nullptr;
            d.nops = ps.op_end - ps.op_begin;
            d.n = n;
            d.nterms = (int32_t)c->ox.size();
            rd.push_back(d);
        }
        if ((r = upload_vec(&G.hres, rd)) != PP_OK) return r;
    } else {
        std::vector<pp::TilePassDesc> td;
        for (const pp::DensePass &ps : P.heis.passes) {
            pp::TilePassDesc d{};
            d.coef = c->coef;
            d.ops = G.hops;
            d.maps = G.hmaps;
            d.n = n;
            d.k = k_heis;
            d.op_begin = ps.op_begin;
            d.op_end = ps.op_end;
            d.ntiles = (int)((int64_t)1 << (2 * (n - k_heis)));
            for (int j = 0; j < k_heis; ++j) d.qubits |= (uint64_t)ps.qubit[j] << (8 * j);
            d.reg_entry = pp::pass_reg_entry(P.heis, ps);
            td.push_back(d);
        }
        if ((r = upload_vec(&G.hpass, td)) != PP_OK) return r;
    }
    HIPCHK(dalloc(&G.ckpt, (size_t)slots * std::max<size_t>(S, 1)));
    HIPCHK(dalloc(&G.rbuf, (size_t)slots));
    const int ntiles_f = (int)((int64_t)1 << (2 * (n - k_fwd)));
    int max_seg = 1;
    for (size_t sg = 0; sg < S; ++sg) max_seg = std::max(max_seg, P.seg_slot_begin[sg + 1] - P.seg_slot_begin[sg]);
    HIPCHK(dalloc(&G.partials, (size_t)max_seg * ntiles_f));
    HIPCHK(dalloc(&G.rot_grad, (size_t)std::max<size_t>(P.slot_param.size(), 1)));
    std::vector<pp::GradPassDesc> gd;
    for (size_t sg = 0; sg < S; ++sg)
        for (int p = P.fwd_pass_begin[sg]; p < P.fwd_pass_begin[sg + 1]; ++p) {
            const pp::DensePass &ps = P.fwd.passes[p];
            pp::GradPassDesc d{};
            d.c = (double *)c->coef;
            d.r = G.rbuf;
            d.ops = G.fops;
            d.maps = G.fmaps;
            d.partials = G.partials;
            d.n = n;
            d.k = k_fwd;
            d.op_begin = ps.op_begin;
            d.op_end = ps.op_end;
            d.ntiles = ntiles_f;
            d.slot_base = P.seg_slot_begin[sg];
            for (int j = 0; j < k_fwd; ++j) d.qubits |= (uint64_t)ps.qubit[j] << (8 * j);
            gd.push_back(d);
        }
    if ((r = upload_vec(&G.gpass, gd)) != PP_OK) return r;
    G.k_heis = k_heis;
    G.k_fwd = k_fwd;
    G.every = every;
    G.valid = true;
    return PP_OK;
}

}  // namespace

// ================================================================ sweeps
// <O> at `count` parameter vectors of one DENSE circuit in shared launches:
// every set has its own maps and weights, all sets share the schedule, so a
// pass of all of them is one launch (and LDS-resident circuits one launch).
extern "C" pp_status pp_evaluate_thetas(pp_circuit *c, int64_t count, const double *thetas, int32_t on_device,
                                        void *stream, double *d_expvals) {
    if (!c) return fail(PP_ERR_INVALID, "null circuit");
    if (count < 0 || (count > 0 && (!thetas || !d_expvals))) return fail(PP_ERR_INVALID, "bad sweep arguments");
    if (count == 0) return PP_OK;
    if (count > (1 << 20)) return fail(PP_ERR_INVALID, "at most 2^20 parameter sets per sweep");
    if (!c->have_gates) return fail(PP_ERR_STATE, "gates not loaded");
    if (!c->have_obs) return fail(PP_ERR_STATE, "observable not set");
    if (c->engine != PP_ENGINE_DENSE || c->track || c->ramp_opt)
        return fail(PP_ERR_STATE, "parameter sweeps run on the DENSE engine without term tracking or frame ramp");
    hipStream_t s = (hipStream_t)stream;
    pp_status r = ensure_plan(c);
    if (r != PP_OK) return r;
    fill_plan_stats(c);
    const pp::DensePlan &P = c->dplan;
    auto &W = c->sw;
    const int64_t np = std::max<int64_t>(c->g.n_params, 1);
    const int64_t nm = std::max(P.nmaps(), 1);
    const int64_t slots = dense_slots(c->n);
    if (count > W.cap || W.gen != c->plan_gen) {
        HIPCHK(hipStreamSynchronize(s));
        if (W.gen != c->plan_gen || count > W.cap) free_sweep(c);
        const int64_t cap = count;
        hipError_t e = dalloc(&W.thetas, (size_t)(np * cap));
        if (e == hipSuccess) e = dalloc(&W.maps, (size_t)(9 * nm * cap));
        if (e == hipSuccess && !P.resident) e = dev_alloc(&W.coef, (size_t)slots * c->dbytes * cap);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            free_sweep(c);
            return fail(PP_ERR_NOMEM, "sweep buffers for " + std::to_string(count) + " parameter sets");
        }
        W.cap = cap;
        W.gen = c->plan_gen;
        W.count = -1;
    }
    if (c->g.n_params > 0)
        HIPCHK(hipMemcpyAsync(W.thetas, thetas, sizeof(double) * c->g.n_params * count,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    if (W.count != count || W.out != d_expvals) {
        // descriptors: compose jobs, then resident jobs or every pass's jobs
        std::vector<unsigned char> blob;
        auto append = [&](const void *p, size_t bytes) {
            const size_t off = blob.size();
            blob.resize(off + ((bytes + 255) & ~size_t(255)));
            std::memcpy(blob.data() + off, p, bytes);
            return off;
        };
        std::vector<pp::ComposeDesc> comp(count);
        for (int64_t i = 0; i < count; ++i) {
            comp[i] = c->h_comp;
            comp[i].theta = W.thetas + i * np;
            comp[i].maps = W.maps + i * nm * 9;
        }
        W.comp_off = append(comp.data(), comp.size() * sizeof(comp[0]));
        if (P.resident) {
            std::vector<pp::ResidentDesc> rd(count);
            for (int64_t i = 0; i < count; ++i) {
                rd[i] = c->h_res;
                rd[i].maps = W.maps + i * nm * 9;
                rd[i].expval_out = d_expvals + i;
                rd[i].coef_out = nullptr;
                rd[i].pres_out = nullptr;
                rd[i].counters = nullptr;
            }
            W.res_off = append(rd.data(), rd.size() * sizeof(rd[0]));
        } else {
            std::vector<pp::TilePassDesc> td;
            td.reserve((size_t)count * P.passes.size());
            for (size_t l = 0; l < P.passes.size(); ++l)
                for (int64_t i = 0; i < count; ++i) {
                    pp::TilePassDesc d = c->h_pass[l];
                    d.coef = (unsigned char *)W.coef + (size_t)i * slots * c->dbytes;
                    d.maps = W.maps + i * nm * 9;
                    d.tile_begin = (int32_t)(i * d.ntiles);
                    td.push_back(d);
                }
            W.pass_off = td.empty() ? 0 : append(td.data(), td.size() * sizeof(td[0]));
        }
        if (blob.size() > W.dcap) {
            HIPCHK(hipStreamSynchronize(s));
            dfree(W.dbuf);
            W.dcap = 0;
            HIPCHK(dev_alloc(&W.dbuf, blob.size()));
            W.dcap = blob.size();
        }
        r = W.staging.upload(W.dbuf, blob.data(), blob.size(), s);
        if (r != PP_OK) return r;
        W.count = count;
        W.out = d_expvals;
    }
    unsigned char *base = (unsigned char *)W.dbuf;
    if (P.nmaps() > 0) {
        ProfScope ps(PC_COMPOSE, s);
        HIPCHK(pp::launch_compose((const pp::ComposeDesc *)(base + W.comp_off), (int)count, s, P.nmaps()));
    }
    if (P.resident) {
        ProfScope ps(PC_RES, s);
        HIPCHK(pp::launch_resident((const pp::ResidentDesc *)(base + W.res_off), (int)count, c->n, c->dbytes, false,
                                   s));
        return PP_OK;
    }
    {
        ProfScope ps(PC_INIT, s);
        HIPCHK(pp::launch_dense_init(W.coef, nullptr, c->n, c->dbytes, c->d_ox, c->d_oz, c->d_oc, (int)c->ox.size(),
                                     s, (int)count));
    }
    const int shift = 2 * (c->n - P.k);
    const int64_t ntiles = (int64_t)1 << shift;
    if (count * ntiles > INT32_MAX) return fail(PP_ERR_INVALID, "too many tiles in one sweep launch");
    TileSpan span;
    span.begin(s);
    for (size_t l = 0; l < P.passes.size(); ++l) {
        // one launch: the sets' descriptors of pass l are consecutive
        pp::TileGroups grp{};
        grp.ngroups = 1;
        grp.first_block[0] = 0;
        grp.first_block[1] = (int32_t)(count * ntiles);
        grp.first_desc[0] = 0;
        grp.shift[0] = shift;
        HIPCHK(pp::launch_tile_pass((const pp::TilePassDesc *)(base + W.pass_off) + l * count, grp, P.k, c->dbytes,
                                    false, s));
        span.count();
    }
    span.end();
    {
        ProfScope ps(PC_READOUT, s);
        HIPCHK(pp::launch_dense_readout(W.coef, c->n, c->dbytes, d_expvals, s, (int)count));
    }
    return PP_OK;
}

pp_status enqueue_gradient_body(pp_circuit *c, hipStream_t s, double *d_expval, double *d_grad);

extern "C" pp_status pp_gradient(pp_circuit *c, void *stream, int32_t checkpoint_every_gates, double *d_expval,
                                 double *d_grad) {
    pp_status r = check_ready(c);
    if (r != PP_OK) return r;
    if (!d_expval || (c->g.n_params > 0 && !d_grad)) return fail(PP_ERR_INVALID, "null output");
    if (checkpoint_every_gates < 0) return fail(PP_ERR_INVALID, "checkpoint_every_gates must be >= 0");
    if (c->engine != PP_ENGINE_DENSE) return fail(PP_ERR_INVALID, "pp_gradient needs the DENSE engine");
    if (c->dtype != PP_F64) return fail(PP_ERR_INVALID, "pp_gradient needs FP64 weights");
    if ((r = ensure_plan(c)) != PP_OK) return r;
    const int64_t every = checkpoint_every_gates > 0 ? checkpoint_every_gates : 256;
    if ((r = ensure_grad(c, every)) != PP_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    auto &G = c->gr;
    if (c->use_graph) {
        const int np = c->g.n_params;
        if (!G.gexec) {
            HIPCHK(dalloc(&G.out, (size_t)1 + np));
            hipStream_t cs;
            HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                g_prof.capturing++;
                r = enqueue_gradient_body(c, cs, G.out, G.out + 1);
                g_prof.capturing--;
                hipGraph_t gr = nullptr;
                hipError_t e2 = hipStreamEndCapture(cs, &gr);
                if (r == PP_OK && e2 == hipSuccess) {
                    G.graph = gr;
                    e2 = hipGraphInstantiate(&G.gexec, gr, nullptr, nullptr, 0);
                }
                if (e2 != hipSuccess && r == PP_OK) r = fail(PP_ERR_DEVICE, "gradient graph capture failed");
            } else {
                r = fail(PP_ERR_DEVICE, "hipStreamBeginCapture failed");
            }
            (void)hipStreamDestroy(cs);
            if (r != PP_OK) {
                free_grad_graph(c);
                return r;
            }
        }
        HIPCHK(hipGraphLaunch(G.gexec, s));
        HIPCHK(pp::launch_copy_f64(G.out, d_expval, 1, s));
        if (np > 0) HIPCHK(pp::launch_copy_f64(G.out + 1, d_grad, np, s));
    } else {
        if ((r = enqueue_gradient_body(c, s, d_expval, d_grad)) != PP_OK) return r;
    }
    fill_plan_stats(c);
    c->evaluated = false;  // the dense weights now hold the forward-swept set
    return PP_OK;
}

// Parameter-shift gradient (the rule of Sec. I: a rotation's derivative is
// half the difference of two evaluations at its angle +- pi/2), as one
// parameter sweep over 2R shifted sets of a private circuit in which every
// rotation gate has a parameter of its own.
extern "C" pp_status pp_psr_gradient(pp_circuit *c, void *stream, double *d_grad) {
    pp_status r = check_ready(c);
    if (r != PP_OK) return r;
    if (c->g.n_params > 0 && !d_grad) return fail(PP_ERR_INVALID, "d_grad is NULL");
    if (c->engine != PP_ENGINE_DENSE || c->track)
        return fail(PP_ERR_STATE, "pp_psr_gradient runs on the DENSE engine without term tracking");
    hipStream_t s = (hipStream_t)stream;
    const int np = c->g.n_params;
    int R = 0;
    for (int64_t g = 0; g < c->g.m; ++g) R += c->g.op[(size_t)g] >= PP_RX;
    if ((int64_t)2 * R * R > ((int64_t)1 << 27))
        return fail(PP_ERR_CAPACITY, "parameter-shift sweep over " + std::to_string(R) + " rotations is too large");
    if (np == 0) return PP_OK;
    if (R == 0) {
        HIPCHK(hipMemsetAsync(d_grad, 0, sizeof(double) * np, s));
        return PP_OK;
    }
    if (!c->psr || c->psr_gen != c->gates_gen || c->psr_obs_gen != c->obs_gen) {
        if (c->psr) pp_circuit_destroy(c->psr);
        c->psr = nullptr;
        dfree(c->d_psr_rot_param);
        dfree(c->d_psr_off);
        dfree(c->d_psr_rot);
        dfree(c->d_psr_thetas);
        dfree(c->d_psr_vals);
        const int64_t m = c->g.m;
        std::vector<int32_t> pexp((size_t)m, 0), rot_param;
        std::vector<std::vector<int32_t>> by_param((size_t)np);
        for (int64_t g = 0; g < m; ++g)
            if (c->g.op[(size_t)g] >= PP_RX) {
                const int32_t j = (int32_t)rot_param.size();
                pexp[(size_t)g] = j;
                rot_param.push_back(c->g.param[(size_t)g]);
                by_param[(size_t)c->g.param[(size_t)g]].push_back(j);
            }
        std::vector<int32_t> off(1, 0), rots;
        for (auto &v : by_param) {
            rots.insert(rots.end(), v.begin(), v.end());
            off.push_back((int32_t)rots.size());
        }
        pp_circuit *a = nullptr;
        if ((r = pp_circuit_create(c->n, c->dtype, PP_ENGINE_DENSE, &a)) != PP_OK) return r;
        r = pp_circuit_load_gates(a, m, c->g.op.data(), c->g.q0.data(), c->g.q1.data(), pexp.data(), R);
        if (r == PP_OK) r = pp_circuit_set_observable(a, (int64_t)c->ox.size(), c->ox.data(), c->oz.data(), c->oc.data());
        if (r == PP_OK && c->tile_opt) r = pp_circuit_set_option(a, PP_OPT_TILE_QUBITS, c->tile_opt);
        if (r == PP_OK) r = upload_vec(&c->d_psr_rot_param, rot_param);
        if (r == PP_OK) r = upload_vec(&c->d_psr_off, off);
        if (r == PP_OK) r = upload_vec(&c->d_psr_rot, rots);
        if (r == PP_OK && dalloc(&c->d_psr_thetas, (size_t)2 * R * R) != hipSuccess)
            r = fail(PP_ERR_NOMEM, "parameter-shift sets");
        if (r == PP_OK && dalloc(&c->d_psr_vals, (size_t)2 * R) != hipSuccess)
            r = fail(PP_ERR_NOMEM, "parameter-shift results");
        if (r != PP_OK) {
            pp_circuit_destroy(a);
            return r;
        }
        c->psr = a;
        c->psr_gen = c->gates_gen;
        c->psr_obs_gen = c->obs_gen;
        c->psr_R = R;
    }
    const long long total = 2ll * R * R;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(psr_thetas_kernel, dim3(blocks), dim3(256), 0, s, c->d_theta, c->d_psr_rot_param, R,
                       c->d_psr_thetas);
    HIPCHK(hipGetLastError());
    if ((r = pp_evaluate_thetas(c->psr, 2 * R, c->d_psr_thetas, 1, stream, c->d_psr_vals)) != PP_OK) return r;
    hipLaunchKernelGGL(psr_combine_kernel, dim3((np + 255) / 256), dim3(256), 0, s, c->d_psr_vals, c->d_psr_off,
                       c->d_psr_rot, np, d_grad);
    HIPCHK(hipGetLastError());
    return PP_OK;
}

// The launch sequence of one gradient (no host synchronization and no
// memsets, so it can be captured in a graph; theta is read from device
// memory by the compose launch).
pp_status enqueue_gradient_body(pp_circuit *c, hipStream_t s, double *d_expval, double *d_grad) {
    auto &G = c->gr;
    const pp::GradPlan &P = G.plan;
    const int n = c->n;
    const size_t S = P.bounds.size() - 1;
    const int64_t slots = dense_slots(n);
    double *coef = (double *)c->coef;
    if (G.ncomp > 0) {
        ProfScope ps(PC_COMPOSE, s);
        HIPCHK(pp::launch_compose(G.comp, G.ncomp, s, std::max(P.heis.nmaps(), P.fwd.nmaps())));
    }
    // Heisenberg sweep, last segment first; checkpoint c(O_b) at every
    // segment start b
    for (size_t sg = S; sg-- > 0;) {
        if (P.heis.resident) {
            ProfScope ps(PC_RES, s);
            HIPCHK(pp::launch_resident(G.hres + sg, 1, n, 8, false, s));
        } else {
            if (sg + 1 == S) {
                ProfScope ps(PC_INIT, s);
                HIPCHK(pp::launch_dense_init(c->coef, nullptr, n, 8, c->d_ox, c->d_oz, c->d_oc, (int)c->ox.size(), s));
            }
            const int shift = 2 * (n - G.k_heis);
            TileSpan span;
            span.begin(s);
            for (int p = P.heis_pass_begin[sg]; p < P.heis_pass_begin[sg + 1]; ++p) {
                pp::TileGroups grp{};
                grp.ngroups = 1;
                grp.first_block[1] = 1 << shift;
                grp.first_desc[0] = p;
                grp.shift[0] = shift;
                HIPCHK(pp::launch_tile_pass(G.hpass, grp, G.k_heis, 8, false, s));
                span.count();
            }
            span.end();
        }
        if (sg > 0) HIPCHK(pp::launch_copy_f64(coef, G.ckpt + (size_t)sg * slots, slots, s));
    }
    {
        ProfScope ps(PC_READOUT, s);
        HIPCHK(pp::launch_dense_readout(c->coef, n, 8, d_expval, s));
    }
    // forward sweep of (c, r) with the joins of every rotation
    HIPCHK(pp::launch_grad_init_state(G.rbuf, n, s));
    const int ntiles_f = (int)((int64_t)1 << (2 * (n - G.k_fwd)));
    int gp = 0;
    for (size_t sg = 0; sg < S; ++sg) {
        if (sg > 0) HIPCHK(pp::launch_copy_f64(G.ckpt + (size_t)sg * slots, coef, slots, s));
        for (int p = P.fwd_pass_begin[sg]; p < P.fwd_pass_begin[sg + 1]; ++p, ++gp) {
            ProfScope ps(PC_TILE, s);
            HIPCHK(pp::launch_grad_pass(G.gpass + gp, ntiles_f, G.k_fwd, s));
        }
        const int nsl = P.seg_slot_begin[sg + 1] - P.seg_slot_begin[sg];
        HIPCHK(pp::launch_grad_reduce(G.partials, nsl, ntiles_f, G.rot_grad + P.seg_slot_begin[sg], s));
    }
    if (c->g.n_params > 0)
        HIPCHK(pp::launch_grad_accumulate(G.rot_grad, G.slot_param, (int)P.slot_param.size(), d_grad, c->g.n_params,
                                          s));
    return PP_OK;
}

extern "C" pp_status pp_profile_enable(int32_t on) {
    g_prof.on = on != 0;
    return PP_OK;
}

extern "C" pp_status pp_profile_read(pp_kernel_time *out, int32_t max, int32_t *n_out) {
    if (!n_out || (max > 0 && !out)) return fail(PP_ERR_INVALID, "null argument");
    double ms[PC_N] = {0};
    int64_t cnt[PC_N] = {0};
    for (const auto &r : g_prof.recs) {
        HIPCHK(hipEventSynchronize(g_prof.pool[r.start + 1]));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, g_prof.pool[r.start], g_prof.pool[r.start + 1]));
        ms[r.cls] += t;
        cnt[r.cls] += r.launches;
    }
    g_prof.recs.clear();
    g_prof.used = 0;
    int k = 0;
    for (int c = 0; c < PC_N; ++c) {
        if (!cnt[c]) continue;
        if (k < max) {
            std::memset(out[k].name, 0, sizeof(out[k].name));
            std::strncpy(out[k].name, kProfNames[c], sizeof(out[k].name) - 1);
            out[k].launches = cnt[c];
            out[k].total_ms = ms[c];
        }
        ++k;
    }
    *n_out = std::min(k, max);
    return PP_OK;
}

// ================================================================= serving
namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int64_t footprint_bytes(const pp_circuit *c) {
    if (c->engine == PP_ENGINE_DENSE) return dense_slots(c->n) * c->dbytes;
    const int64_t cap = c->max_terms > 0 ? c->max_terms : (c->n <= 12 ? dense_slots(c->n) : ((int64_t)1 << 24));
    return 2 * cap * (16 + 2 * (int64_t)c->dbytes);
}

enum ReqState { RQ_PREP = 0, RQ_QUEUED, RQ_ACTIVE, RQ_FINISHING, RQ_DONE };

struct ServedReq {
    int64_t ticket = 0;
    pp_circuit *c = nullptr;
    std::atomic<int> state{RQ_PREP};  // written by the serving thread, read by pp_server_poll
    bool resident = false;  // runs whole in one LDS-resident launch
    bool pooled = false;    // tiled DENSE: weights in a buffer of the server's pool
    void *buf = nullptr;    // the pool buffer while active
    int64_t foot = 0;       // bytes counted against the budget while active
    double t_submit = 0, t_done = 0;
    size_t pass = 0;
    int slot = -1;
    hipEvent_t ev = nullptr;
    double result = 0;
    pp_status status = PP_OK;
};

constexpr int kRing = 4;
// LDS-resident requests run whole, batched per launch, on a few streams of
// their own beside the tile passes (kernels of one stream run in order, so a
// single side stream would serialize one-workgroup launches)
constexpr int kSideLanes = 3;
// host threads that plan admitted-to-be requests (planning a 60k-gate
// circuit takes tens of milliseconds of host time)
constexpr int kPrepThreads = 4;

}  // namespace

struct pp_server {
    std::mutex mu;
    std::condition_variable cv, done_cv, prep_cv;
    std::thread th;
    std::vector<std::thread> preps;
    bool stop = false;
    std::deque<ServedReq *> prep_queue;  // submitted, waiting for a preparation thread
    int preparing = 0;                   // being prepared
    std::deque<ServedReq *> queue;       // prepared, waiting for admission (ticket order)
    std::vector<ServedReq *> active;
    std::unordered_map<int64_t, ServedReq *> reqs;
    std::unordered_set<const pp_circuit *> live;  // circuits submitted and not done
    int64_t next_ticket = 1;
    int64_t budget = 0, used = 0;
    int64_t max_queued = 0;  // 0: no limit
    int max_active = 0;
    hipStream_t main = nullptr, side = nullptr;
    double *d_results = nullptr, *h_results = nullptr;
    std::vector<int> free_slots;
    // weight buffers of tiled requests: returned at completion and reused;
    // held (in use + free) never exceeds the budget
    std::multimap<size_t, void *> pool_free;
    int64_t pool_held = 0, pool_peak = 0;
    struct Ring {
        void *d = nullptr, *h = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool used = false;
    } ring[kRing];
    int ring_i = 0;
    struct SideLane {
        hipStream_t st = nullptr;
        void *d = nullptr, *h = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool busy = false;
    } lane[kSideLanes];
    std::vector<ServedReq *> res_pending;
    int64_t iterations = 0, tile_launches = 0, max_in_flight = 0, resident_launches = 0;
    int dev = 0;
};

namespace {

pp_status ring_upload(pp_server *S, const std::vector<unsigned char> &blob, void **dptr) {
    pp_server::Ring &R = S->ring[S->ring_i];
    S->ring_i = (S->ring_i + 1) % kRing;
    if (R.used) HIPCHK(hipEventSynchronize(R.ev));  // bounds how far the host runs ahead
    if (blob.size() > R.cap) {
        dev_free(R.d);
        if (R.h) (void)hipHostFree(R.h);
        R.d = R.h = nullptr;
        R.cap = 0;
        const size_t cap = std::max<size_t>(blob.size() * 2, 1 << 16);
        HIPCHK(dev_alloc(&R.d, cap));
        HIPCHK(hipHostMalloc(&R.h, cap, hipHostMallocDefault));
        R.cap = cap;
    }
    std::memcpy(R.h, blob.data(), blob.size());
    HIPCHK(hipMemcpyAsync(R.d, R.h, blob.size(), hipMemcpyHostToDevice, S->main));
    if (!R.ev) HIPCHK(hipEventCreateWithFlags(&R.ev, hipEventDisableTiming));
    *dptr = R.d;
    return PP_OK;
}

void ring_mark(pp_server *S) {
    pp_server::Ring &R = S->ring[(S->ring_i + kRing - 1) % kRing];
    if (hipEventRecord(R.ev, S->main) == hipSuccess) R.used = true;
}

// A weight buffer of `bytes` from the pool: a free one of that size, else a
// new one, after returning free buffers of other sizes while the pool would
// exceed the budget.  Admission keeps the active footprints within the
// budget, so the free buffers always cover the difference.
pp_status pool_take(pp_server *S, size_t bytes, void **out) {
    auto it = S->pool_free.find(bytes);
    if (it != S->pool_free.end()) {
        *out = it->second;
        S->pool_free.erase(it);
        return PP_OK;
    }
    while (S->pool_held + (int64_t)bytes > S->budget && !S->pool_free.empty()) {
        auto big = std::prev(S->pool_free.end());
        dev_free(big->second);
        S->pool_held -= (int64_t)big->first;
        S->pool_free.erase(big);
    }
    void *p = nullptr;
    HIPCHK(dev_alloc(&p, bytes));
    S->pool_held += (int64_t)bytes;
    S->pool_peak = std::max(S->pool_peak, S->pool_held);
    *out = p;
    return PP_OK;
}

pp_status finish_async(pp_server *S, ServedReq *r, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(S->h_results + r->slot, S->d_results + r->slot, sizeof(double), hipMemcpyDeviceToHost, st));
    if (!r->ev) HIPCHK(hipEventCreateWithFlags(&r->ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(r->ev, st));
    r->state = RQ_FINISHING;
    return PP_OK;
}

// Orders the work about to be issued on `st` after the request's theta upload
// (made by the caller on a stream of its own before pp_server_submit).
pp_status after_theta(const pp_circuit *c, hipStream_t st) {
    if (c->theta_ev) HIPCHK(hipStreamWaitEvent(st, c->theta_ev, 0));
    return PP_OK;
}

// Preparation, on a preparation thread: the schedule is built and uploaded
// (the circuit's own 4^n weights are not allocated for DENSE circuits
// without term tracking: tiled ones run in pool buffers, LDS-resident ones
// need none).
pp_status prepare_request(ServedReq *r) {
    pp_circuit *c = r->c;
    const bool dense_fast = c->engine == PP_ENGINE_DENSE && !c->track && !ramp_wanted(c);
    pp_status st = ensure_plan(c, !dense_fast);
    if (st != PP_OK) return st;
    fill_plan_stats(c);
    r->resident = dense_fast && c->dplan.resident;
    r->pooled = dense_fast && !c->dplan.resident;
    r->foot = r->resident ? 0 : footprint_bytes(c);
    return PP_OK;
}

// Starts an admitted request: the whole evaluation for requests outside the
// batched paths; maps and start weights for tiled ones.
pp_status start_request(pp_server *S, ServedReq *r) {
    pp_circuit *c = r->c;
    double *out = S->d_results + r->slot;
    if (r->resident) return PP_OK;  // launched with the other pending resident requests
    if (!r->pooled) {
        pp_status st = after_theta(c, S->side);
        if (st == PP_OK) st = pp_evaluate(c, S->side, out);
        if (st != PP_OK) return st;
        return finish_async(S, r, S->side);
    }
    pp_status st = pool_take(S, (size_t)r->foot, &r->buf);
    if (st != PP_OK) return st;
    if ((st = after_theta(c, S->main)) != PP_OK) return st;
    if (c->dplan.nmaps() > 0) HIPCHK(pp::launch_compose(c->d_comp, 1, S->main, c->dplan.nmaps()));
    HIPCHK(pp::launch_dense_init(r->buf, nullptr, c->n, c->dbytes, c->d_ox, c->d_oz, c->d_oc, (int)c->ox.size(),
                                 S->main));
    r->pass = 0;
    return PP_OK;
}

// Launches every pending resident request on an idle side lane: the maps of
// all of them in one compose launch, then one resident launch per (dtype, n)
// with one workgroup per request.  Does nothing while every lane is busy.
pp_status launch_resident_batch(pp_server *S, bool *launched) {
    *launched = false;
    pp_server::SideLane *Ln = nullptr;
    for (auto &cand : S->lane) {
        if (cand.busy && hipEventQuery(cand.ev) == hipSuccess) cand.busy = false;
        if (!cand.busy) {
            Ln = &cand;
            break;
        }
    }
    if (!Ln) return PP_OK;
    std::vector<ServedReq *> &P = S->res_pending;
    std::stable_sort(P.begin(), P.end(), [](ServedReq *a, ServedReq *b) {
        return a->c->dbytes != b->c->dbytes ? a->c->dbytes > b->c->dbytes : a->c->n > b->c->n;
    });
    std::vector<pp::ComposeDesc> comp;
    int comp_max = 1;
    for (ServedReq *r : P)
        if (r->c->dplan.nmaps() > 0) {
            comp.push_back(r->c->h_comp);
            comp_max = std::max(comp_max, r->c->dplan.nmaps());
        }
    std::vector<pp::ResidentDesc> rd;
    for (ServedReq *r : P) {
        pp::ResidentDesc d = r->c->h_res;
        d.expval_out = S->d_results + r->slot;
        rd.push_back(d);
    }
    const size_t cbytes = comp.size() * sizeof(pp::ComposeDesc);
    const size_t roff = (cbytes + 255) & ~(size_t)255;
    const size_t bytes = roff + rd.size() * sizeof(pp::ResidentDesc);
    if (bytes > Ln->cap) {  // the lane is idle: its buffers are free
        dev_free(Ln->d);
        if (Ln->h) (void)hipHostFree(Ln->h);
        Ln->d = Ln->h = nullptr;
        Ln->cap = 0;
        const size_t cap = std::max<size_t>(2 * bytes, 1 << 16);
        HIPCHK(dev_alloc(&Ln->d, cap));
        HIPCHK(hipHostMalloc(&Ln->h, cap, hipHostMallocDefault));
        Ln->cap = cap;
    }
    for (ServedReq *r : P) {
        pp_status st = after_theta(r->c, Ln->st);
        if (st != PP_OK) return st;
    }
    if (!comp.empty()) std::memcpy(Ln->h, comp.data(), cbytes);
    std::memcpy((unsigned char *)Ln->h + roff, rd.data(), rd.size() * sizeof(pp::ResidentDesc));
    HIPCHK(hipMemcpyAsync(Ln->d, Ln->h, bytes, hipMemcpyHostToDevice, Ln->st));
    if (!comp.empty()) HIPCHK(pp::launch_compose((const pp::ComposeDesc *)Ln->d, (int)comp.size(), Ln->st, comp_max));
    const pp::ResidentDesc *dres = (const pp::ResidentDesc *)((unsigned char *)Ln->d + roff);
    size_t i = 0;
    while (i < P.size()) {
        size_t j = i;
        while (j < P.size() && P[j]->c->n == P[i]->c->n && P[j]->c->dbytes == P[i]->c->dbytes) ++j;
        HIPCHK(pp::launch_resident(dres + i, (int)(j - i), P[i]->c->n, P[i]->c->dbytes, false, Ln->st));
        S->resident_launches++;
        i = j;
    }
    for (ServedReq *r : P) {
        pp_status st = finish_async(S, r, Ln->st);
        if (st != PP_OK) return st;
    }
    if (!Ln->ev) HIPCHK(hipEventCreateWithFlags(&Ln->ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(Ln->ev, Ln->st));
    Ln->busy = true;
    P.clear();
    *launched = true;
    return PP_OK;
}

// Marks a request done (caller holds S->mu).  A tiled request's pool buffer
// goes back to the pool: its last use (the readout) came before the event
// that completed it, and a failed request has nothing left in flight on it
// once the server stream it used has been synchronized by the caller.
void complete(pp_server *S, ServedReq *r, pp_status st) {
    r->status = st;
    r->t_done = now_s();
    if (st == PP_OK) r->result = S->h_results[r->slot];
    r->state = RQ_DONE;
    pp_circuit *c = r->c;
    if (r->buf) {
        S->pool_free.emplace((size_t)r->foot, r->buf);
        r->buf = nullptr;
    }
    // a pooled run keeps no final weights with the circuit
    c->evaluated = !r->pooled && !r->resident && st == PP_OK;
    c->last_track = c->track;
    S->live.erase(c);
}

bool server_idle(const pp_server *S) {
    return S->prep_queue.empty() && S->preparing == 0 && S->queue.empty() && S->active.empty();
}

void prep_loop(pp_server *S) {
    (void)hipSetDevice(S->dev);
    for (;;) {
        ServedReq *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->prep_cv.wait(lk, [&] { return S->stop || !S->prep_queue.empty(); });
            if (S->prep_queue.empty()) return;  // stopping, nothing left
            r = S->prep_queue.front();
            S->prep_queue.pop_front();
            S->preparing++;
        }
        const pp_status st = prepare_request(r);
        std::lock_guard<std::mutex> lk(S->mu);
        S->preparing--;
        if (st != PP_OK) {
            complete(S, r, st);
            S->done_cv.notify_all();
        } else {
            r->state = RQ_QUEUED;
            auto pos = std::upper_bound(S->queue.begin(), S->queue.end(), r,
                                        [](const ServedReq *a, const ServedReq *b) { return a->ticket < b->ticket; });
            S->queue.insert(pos, r);
        }
        S->cv.notify_all();
    }
}

void server_loop(pp_server *S) {
    (void)hipSetDevice(S->dev);
    std::vector<ServedReq *> fresh;
    for (;;) {
        fresh.clear();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop && server_idle(S)) break;
            // admission in ticket order among the prepared requests
            while (!S->queue.empty() && (int)S->active.size() < S->max_active && !S->free_slots.empty()) {
                ServedReq *r = S->queue.front();
                if (S->used + r->foot > S->budget && !S->active.empty()) break;  // wait for memory
                S->queue.pop_front();
                S->used += r->foot;
                r->slot = S->free_slots.back();
                S->free_slots.pop_back();
                r->state = RQ_ACTIVE;
                S->active.push_back(r);
                fresh.push_back(r);
            }
            S->max_in_flight = std::max<int64_t>(S->max_in_flight, (int64_t)S->active.size());
            if (S->active.empty()) {
                // nothing in flight: sleep until a prepared request is queued
                // (a preparation thread notifies) or the server stops
                S->cv.wait(lk, [&] {
                    return !S->queue.empty() || (S->stop && S->prep_queue.empty() && S->preparing == 0);
                });
                continue;
            }
        }
        for (ServedReq *r : fresh) {
            pp_status st = start_request(S, r);
            if (st != PP_OK) {
                (void)hipStreamSynchronize(S->main);
                (void)hipStreamSynchronize(S->side);
                std::lock_guard<std::mutex> lk(S->mu);
                complete(S, r, st);
            } else if (r->resident) {
                S->res_pending.push_back(r);
            }
        }
        if (!S->res_pending.empty()) {
            bool res_launched = false;
            std::vector<ServedReq *> batch = S->res_pending;
            pp_status st = launch_resident_batch(S, &res_launched);
            if (st != PP_OK) {
                for (auto &Ln : S->lane) (void)hipStreamSynchronize(Ln.st);
                std::lock_guard<std::mutex> lk(S->mu);
                for (ServedReq *r : batch)
                    if (r->state == RQ_ACTIVE) complete(S, r, st);
                S->res_pending.clear();
            }
        }
        // one iteration: the next pass of every active tiled request, one
        // launch per (tile size, weight type)
        std::vector<ServedReq *> tiled;
        for (ServedReq *r : S->active)
            if (r->state == RQ_ACTIVE && r->pooled) tiled.push_back(r);
        bool launched = false;
        for (int db : {8, 4})
            for (int k = 4; k <= 7 && !tiled.empty(); ++k) {
                std::vector<ServedReq *> grp;
                for (ServedReq *r : tiled)
                    if (r->c->dplan.k == k && r->c->dbytes == db && r->pass < r->c->h_pass.size()) grp.push_back(r);
                if (grp.empty()) continue;
                std::stable_sort(grp.begin(), grp.end(), [](ServedReq *a, ServedReq *b) { return a->c->n > b->c->n; });
                size_t i0 = 0;
                while (i0 < grp.size()) {
                    std::vector<pp::TilePassDesc> td;
                    pp::TileGroups tg{};
                    int run = 0, last_n = -1;
                    size_t i = i0;
                    for (; i < grp.size(); ++i) {
                        pp::TilePassDesc d = grp[i]->c->h_pass[grp[i]->pass];
                        d.coef = grp[i]->buf;
                        if (d.n != last_n) {
                            if (tg.ngroups == pp::kMaxTileGroups) break;
                            tg.first_block[tg.ngroups] = run;
                            tg.first_desc[tg.ngroups] = (int32_t)td.size();
                            tg.shift[tg.ngroups] = 2 * (d.n - k);
                            tg.ngroups++;
                            last_n = d.n;
                        }
                        d.tile_begin = run;
                        run += d.ntiles;
                        td.push_back(d);
                    }
                    tg.first_block[tg.ngroups] = run;
                    std::vector<unsigned char> blob(td.size() * sizeof(pp::TilePassDesc));
                    std::memcpy(blob.data(), td.data(), blob.size());
                    void *dd = nullptr;
                    pp_status st = ring_upload(S, blob, &dd);
                    if (st == PP_OK) {
                        hipError_t e = pp::launch_tile_pass((const pp::TilePassDesc *)dd, tg, k, db, false, S->main);
                        if (e != hipSuccess) st = fail(PP_ERR_DEVICE, hipGetErrorString(e));
                    }
                    ring_mark(S);
                    for (size_t j = i0; j < i; ++j) {
                        ServedReq *r = grp[j];
                        if (st != PP_OK) {
                            (void)hipStreamSynchronize(S->main);
                            std::lock_guard<std::mutex> lk(S->mu);
                            complete(S, r, st);
                            continue;
                        }
                        if (++r->pass == r->c->h_pass.size()) {
                            pp_circuit *c = r->c;
                            if (pp::launch_dense_readout(r->buf, c->n, c->dbytes, S->d_results + r->slot, S->main) !=
                                    hipSuccess ||
                                finish_async(S, r, S->main) != PP_OK) {
                                (void)hipStreamSynchronize(S->main);
                                std::lock_guard<std::mutex> lk(S->mu);
                                complete(S, r, PP_ERR_DEVICE);
                            }
                        }
                    }
                    S->tile_launches++;
                    launched = true;
                    i0 = i;
                }
            }
        // tiled requests with no passes at all (empty circuits)
        for (ServedReq *r : tiled)
            if (r->state == RQ_ACTIVE && r->c->h_pass.empty()) {
                pp_circuit *c = r->c;
                if (pp::launch_dense_readout(r->buf, c->n, c->dbytes, S->d_results + r->slot, S->main) != hipSuccess ||
                    finish_async(S, r, S->main) != PP_OK) {
                    (void)hipStreamSynchronize(S->main);
                    std::lock_guard<std::mutex> lk(S->mu);
                    complete(S, r, PP_ERR_DEVICE);
                }
            }
        if (launched) S->iterations++;
        // completions
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (ServedReq *r : S->active)
                if (r->state == RQ_FINISHING && hipEventQuery(r->ev) == hipSuccess) complete(S, r, PP_OK);
            bool any = false;
            for (size_t i = 0; i < S->active.size();) {
                ServedReq *r = S->active[i];
                if (r->state == RQ_DONE) {
                    S->used -= r->foot;
                    S->free_slots.push_back(r->slot);
                    S->active[i] = S->active.back();
                    S->active.pop_back();
                    any = true;
                } else {
                    ++i;
                }
            }
            if (any) S->done_cv.notify_all();
        }
        if (!launched) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

}  // namespace

extern "C" pp_status pp_server_create(int64_t mem_budget_bytes, int32_t max_active, pp_server **out) {
    if (!out) return fail(PP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (mem_budget_bytes <= 0 || max_active <= 0 || max_active > 4096)
        return fail(PP_ERR_INVALID, "budget must be > 0 and max_active in [1, 4096]");
    pp_server *S = new (std::nothrow) pp_server();
    if (!S) return fail(PP_ERR_NOMEM, "host allocation");
    S->budget = mem_budget_bytes;
    S->max_active = max_active;
    hipError_t e = hipGetDevice(&S->dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->main, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking);
    for (auto &Ln : S->lane)
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&Ln.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = dalloc(&S->d_results, (size_t)max_active);
    if (e == hipSuccess) e = hipHostMalloc((void **)&S->h_results, sizeof(double) * max_active, hipHostMallocDefault);
    if (e != hipSuccess) {
        if (S->main) (void)hipStreamDestroy(S->main);
        if (S->side) (void)hipStreamDestroy(S->side);
        for (auto &Ln : S->lane)
            if (Ln.st) (void)hipStreamDestroy(Ln.st);
        dfree(S->d_results);
        delete S;
        return fail(e == hipErrorOutOfMemory ? PP_ERR_NOMEM : PP_ERR_DEVICE,
                    std::string("server setup: ") + hipGetErrorString(e));
    }
    for (int i = max_active - 1; i >= 0; --i) S->free_slots.push_back(i);
    S->th = std::thread(server_loop, S);
    for (int i = 0; i < kPrepThreads; ++i) S->preps.emplace_back(prep_loop, S);
    *out = S;
    return PP_OK;
}

extern "C" pp_status pp_server_set_queue_limit(pp_server *S, int64_t max_queued) {
    if (!S) return fail(PP_ERR_INVALID, "null server");
    if (max_queued < 0) return fail(PP_ERR_INVALID, "max_queued must be >= 0");
    std::lock_guard<std::mutex> lk(S->mu);
    S->max_queued = max_queued;
    return PP_OK;
}

extern "C" pp_status pp_server_submit(pp_server *S, pp_circuit *c, int64_t *ticket) {
    if (!S || !c || !ticket) return fail(PP_ERR_INVALID, "null argument");
    pp_status r = check_ready(c);
    if (r != PP_OK) return r;
    const int64_t foot = footprint_bytes(c);
    if (foot > S->budget) return fail(PP_ERR_CAPACITY, "request larger than the server memory budget");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(PP_ERR_STATE, "server is shutting down");
    if (S->live.count(c)) return fail(PP_ERR_INVALID, "circuit already submitted and not done");
    if (S->max_queued > 0 && (int64_t)(S->prep_queue.size() + S->preparing + S->queue.size()) >= S->max_queued)
        return fail(PP_ERR_BUSY, "server queue is full");
    ServedReq *q = new (std::nothrow) ServedReq();
    if (!q) return fail(PP_ERR_NOMEM, "host allocation");
    q->c = c;
    q->foot = foot;
    q->ticket = S->next_ticket++;
    q->t_submit = now_s();
    S->live.insert(c);
    S->prep_queue.push_back(q);
    S->reqs[q->ticket] = q;
    *ticket = q->ticket;
    S->prep_cv.notify_one();
    return PP_OK;
}

extern "C" pp_status pp_server_poll(pp_server *S, int64_t ticket, int32_t *done, double *expval, double *latency_us) {
    if (!S || !done) return fail(PP_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(PP_ERR_INVALID, "unknown ticket");
    ServedReq *q = it->second;
    *done = q->state == RQ_DONE;
    if (q->state == RQ_DONE) {
        if (expval) *expval = q->result;
        if (latency_us) *latency_us = (q->t_done - q->t_submit) * 1e6;
        if (q->status != PP_OK) return fail(q->status, "request failed");
    }
    return PP_OK;
}

extern "C" pp_status pp_server_drain(pp_server *S) {
    if (!S) return fail(PP_ERR_INVALID, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    S->done_cv.wait(lk, [&] { return server_idle(S); });
    return PP_OK;
}

extern "C" pp_status pp_server_counters(pp_server *S, int64_t *iterations, int64_t *tile_launches,
                                        int64_t *max_in_flight) {
    if (!S) return fail(PP_ERR_INVALID, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (iterations) *iterations = S->iterations;
    if (tile_launches) *tile_launches = S->tile_launches;
    if (max_in_flight) *max_in_flight = S->max_in_flight;
    return PP_OK;
}

extern "C" pp_status pp_server_pool_bytes(pp_server *S, int64_t *held, int64_t *peak) {
    if (!S) return fail(PP_ERR_INVALID, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (held) *held = S->pool_held;
    if (peak) *peak = S->pool_peak;
    return PP_OK;
}

extern "C" void pp_server_destroy(pp_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
        S->prep_cv.notify_all();
    }
    for (auto &t : S->preps)
        if (t.joinable()) t.join();
    if (S->th.joinable()) S->th.join();
    (void)hipStreamSynchronize(S->main);
    (void)hipStreamSynchronize(S->side);
    for (auto &Ln : S->lane) (void)hipStreamSynchronize(Ln.st);
    for (auto &kv : S->reqs) {
        if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
        delete kv.second;
    }
    for (auto &R : S->ring) {
        if (R.ev) (void)hipEventDestroy(R.ev);
        dev_free(R.d);
        if (R.h) (void)hipHostFree(R.h);
    }
    for (auto &kv : S->pool_free) dev_free(kv.second);
    dfree(S->d_results);
    (void)hipHostFree(S->h_results);
    for (auto &Ln : S->lane) {
        if (Ln.ev) (void)hipEventDestroy(Ln.ev);
        dev_free(Ln.d);
        if (Ln.h) (void)hipHostFree(Ln.h);
        (void)hipStreamDestroy(Ln.st);
    }
    (void)hipStreamDestroy(S->main);
    (void)hipStreamDestroy(S->side);
    delete S;
}

extern "C" pp_status pp_tune_set(pp_tune_key key, int32_t index, int32_t value) {
    if (key == PP_TUNE_TILE_QUBITS) {
        if (index < 8 || index > 16 || value < 4 || value > 7) return fail(PP_ERR_INVALID, "tile qubits: n in 8..16, k in 4..7");
        g_tile_qubits[index] = value;
        return PP_OK;
    }
    if (key == PP_TUNE_TILE_KERNEL) {
        if (index < 4 || index > 7 || value < 0 || value > 4 || (value >= 3 && index != 6) ||
            (index == 7 && value == 2))
            return fail(PP_ERR_INVALID, "tile kernel: k in 4..7, value 0..4 (2: k <= 6; 3, 4: k = 6 only)");
        pp::set_tile_kernel_variant(index, value);
        return PP_OK;
    }
    if (key == PP_TUNE_RESIDENT_BLOCK) {
        if (index < 5 || index > 7 || (value != 256 && value != 512 && value != 1024))
            return fail(PP_ERR_INVALID, "resident block: n in 5..7, value 256/512/1024");
        pp::set_resident_block(index, value);
        return PP_OK;
    }
    if (key == PP_TUNE_SORT_SHAPE) {
        if (index < 0 || index >= pp::kSortClasses || value < 0 || value >= pp::kSortShapeCount)
            return fail(PP_ERR_INVALID, "sort shape: class 0..2, value 0..5");
        pp::set_sort_shape(index, value);
        return PP_OK;
    }
    return fail(PP_ERR_INVALID, "unknown tuning key");
}

extern "C" pp_status pp_tune_get(pp_tune_key key, int32_t index, int32_t *value) {
    if (!value) return fail(PP_ERR_INVALID, "null output");
    if (key == PP_TUNE_TILE_QUBITS && index >= 8 && index <= 16) {
        *value = g_tile_qubits[index];
        return PP_OK;
    }
    if (key == PP_TUNE_TILE_KERNEL && index >= 4 && index <= 7) {
        *value = pp::tile_kernel_variant(index);
        return PP_OK;
    }
    if (key == PP_TUNE_RESIDENT_BLOCK && index >= 5 && index <= 7) {
        *value = pp::resident_block(index);
        return PP_OK;
    }
    if (key == PP_TUNE_SORT_SHAPE && index >= 0 && index < pp::kSortClasses) {
        *value = pp::sort_shape(index);
        return PP_OK;
    }
    return fail(PP_ERR_INVALID, "unknown tuning key or index");
}
