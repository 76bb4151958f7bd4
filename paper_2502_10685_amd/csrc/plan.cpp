// Host planner of libpauliprop.
//
// The observable is propagated in the Heisenberg picture, so gates are taken
// g_m first.  Two schedules are built from the same list:
//
// Dense: the paper divides a circuit into operators of non-CX gates U_k and
// CX gates V_k and groups each U_k by wire, so that all single-qubit gates of
// one wire act as one composed map (Sec. III-A, Sec. III-C, eq. (5)).  Here a
// wire's run of single-qubit gates between two CX gates touching that wire
// becomes one U1 op, whatever other wires do in between (gates on disjoint
// qubits commute).  For n too large for one workgroup's LDS the ops are
// packed into passes over k-qubit tiles: a greedy list scheduler takes every
// gate whose predecessors on its wires are done and whose qubits lie in the
// pass's qubit set, and grows the set (up to k qubits) with the earliest
// ready gate when nothing else fits.
//
// Sparse: one pass per rotation, carrying the Clifford gates that precede it
// (in Heisenberg order), so every Clifford is fused into a rotation's pass.
#include "plan.h"

#include <algorithm>

namespace pp {

// Heisenberg maps on the (X, Y, Z) weights, rows = output letter.
unsigned gate_smask(int op) {
    auto bit = [](int r, int c) { return 1u << (3 * r + c); };
    switch (op) {
    case 0: return bit(0, 2) | bit(1, 1) | bit(2, 0);                                  // H
    case 1: return bit(0, 1) | bit(1, 0) | bit(2, 2);                                  // S
    case 3: return bit(0, 0) | bit(1, 1) | bit(1, 2) | bit(2, 1) | bit(2, 2);          // RX
    case 4: return bit(0, 0) | bit(0, 2) | bit(1, 1) | bit(2, 0) | bit(2, 2);          // RY
    default: return bit(0, 0) | bit(0, 1) | bit(1, 0) | bit(1, 1) | bit(2, 2);         // RZ
    }
}

// boolean product after * before
unsigned smask_compose(unsigned after, unsigned before) {
    unsigned out = 0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            bool v = false;
            for (int t = 0; t < 3; ++t)
                v = v || (((after >> (3 * r + t)) & 1u) && ((before >> (3 * t + c)) & 1u));
            if (v) out |= 1u << (3 * r + c);
        }
    return out;
}

DensePlan plan_dense(const GateList &g, int k, int low, bool compose, bool reorder) {
    PlanOptions o;
    o.compose = compose;
    o.group = compose;
    o.reorder = reorder;
    return plan_dense_opts(g, k, low, o);
}

namespace {

unsigned op_digits(const DOp &d) { return d.kind == DOP_CX ? (1u << d.a) | (1u << d.b) : (1u << d.a); }

}  // namespace

int group_shape(const DOp *m, int count, int lo) {
    if (count < 2 || count > 3 || m[0].kind != DOP_CX) return 0;
    const int dir = m[0].a == lo ? 0 : 1;
    for (int j = 1; j < count; ++j)
        if (m[j].kind != DOP_U1) return 0;
    int code;
    if (count == 2) {
        code = m[1].a == lo ? 0 : 1;
    } else {
        if ((m[1].a == lo) == (m[2].a == lo)) return 0;
        code = m[1].a == lo ? 2 : 3;
    }
    return 1 + 4 * dir + code;
}

namespace {

// A GROUP of one of the eight shapes carries the map indices of its U1
// members in its header (map: the first, reserved: the second, or the
// first again), so a sweep can load its maps as soon as it decodes the
// header.
void set_shape_maps(DOp &h, const DOp *members) {
    if (!h.perm) return;
    h.map = members[1].map;
    h.reserved = h.ngates > 2 ? members[2].map : members[1].map;
}

// Regroups a run of ops: repeatedly takes the first remaining op and every
// later op whose digits stay within one pair of digits and that does not
// share a digit with an op it would move past (ops on disjoint digits
// commute).  Groups of two or more ops get a GROUP header.
std::vector<DOp> group_ops(const std::vector<DOp> &in, int k) {
    std::vector<DOp> out;
    std::vector<char> used(in.size(), 0);
    for (size_t i = 0; i < in.size(); ++i) {
        if (used[i]) continue;
        unsigned pair = op_digits(in[i]), skipped = 0;
        std::vector<size_t> mem{i};
        used[i] = 1;
        for (size_t j = i + 1; j < in.size() && (int)mem.size() < kMaxGroupOps; ++j) {
            if (used[j]) continue;
            const unsigned d = op_digits(in[j]);
            if (d & skipped) {
                skipped |= d;
                continue;
            }
            if (__builtin_popcount(pair | d) <= 2) {
                pair |= d;
                mem.push_back(j);
                used[j] = 1;
            } else {
                skipped |= d;
            }
        }
        if (mem.size() > 1 && __builtin_popcount(pair) == 1) {
            if (k < 2) {  // a one-digit tile has no pair: keep the ops as they are
                for (size_t j : mem) out.push_back(in[j]);
                continue;
            }
            pair |= 1u << (pair == 1u ? 1 : 0);  // any second digit completes the block
        }
        if (mem.size() == 1) {
            out.push_back(in[i]);
            continue;
        }
        DOp h{};
        h.kind = DOP_GROUP;
        h.a = (uint8_t)__builtin_ctz(pair);
        h.b = (uint8_t)(31 - __builtin_clz(pair));
        h.ngates = (uint8_t)mem.size();
        std::vector<DOp> body;
        for (size_t j : mem) body.push_back(in[j]);
        h.perm = (uint16_t)group_shape(body.data(), (int)body.size(), h.a);
        set_shape_maps(h, body.data());
        out.push_back(h);
        out.insert(out.end(), body.begin(), body.end());
    }
    return out;
}

// Orders the ops of a k = kSegTileDigits pass into register segments: the
// same greedy rule as group_ops with up to three digits per segment.  Each
// segment opens with a SEG header naming its digit triple (a < b < smask)
// and the number of entries that follow (GROUP headers included); inside a
// segment ops on a common digit pair are packed into GROUP ops.  A triple
// with spare digits is completed with the previous segment's digits (no
// re-layout between the two) and otherwise with digits 2..5 when the
// segment avoids digits 0 and 1 (a layout that can be loaded from and
// stored to HBM directly).
std::vector<DOp> segment_ops(const std::vector<DOp> &in, int k) {
    std::vector<DOp> out;
    std::vector<char> used(in.size(), 0);
    unsigned prev = 0;
    for (size_t i = 0; i < in.size(); ++i) {
        if (used[i]) continue;
        unsigned set = op_digits(in[i]), skipped = 0;
        std::vector<DOp> mem{in[i]};
        used[i] = 1;
        for (size_t j = i + 1; j < in.size(); ++j) {
            if (used[j]) continue;
            const unsigned d = op_digits(in[j]);
            if (d & skipped) {
                skipped |= d;
                continue;
            }
            if (__builtin_popcount(set | d) <= 3) {
                set |= d;
                mem.push_back(in[j]);
                used[j] = 1;
            } else {
                skipped |= d;
            }
        }
        if (__builtin_popcount(set | prev) == 3) set |= prev;
        const unsigned pref = (set & 3u) ? 0u : 0x3cu;
        for (int q = 0; q < k && __builtin_popcount(set) < 3; ++q)
            if ((pref >> q) & 1u) set |= 1u << q;
        for (int q = 0; q < k && __builtin_popcount(set) < 3; ++q) set |= 1u << q;
        prev = set;
        const std::vector<DOp> body = group_ops(mem, k);
        // SEG headers count at most 255 entries; a GROUP stays with its members
        size_t b = 0;
        while (b < body.size()) {
            size_t e = b;
            while (e < body.size()) {
                const size_t unit = body[e].kind == DOP_GROUP ? 1 + body[e].ngates : 1;
                if (e + unit - b > 255) break;
                e += unit;
            }
            DOp h{};
            h.kind = DOP_SEG;
            h.a = (uint8_t)__builtin_ctz(set);
            h.b = (uint8_t)__builtin_ctz(set & (set - 1));
            h.smask = (uint16_t)(31 - __builtin_clz(set));
            h.ngates = (uint8_t)(e - b);
            out.push_back(h);
            out.insert(out.end(), body.begin() + b, body.begin() + e);
            b = e;
        }
    }
    return out;
}

// Digits an op's LDS sweep covers that matter for the wave split: a lone U1
// on digit a is swept with digit a - 1 (digit 1 for a = 0), which is digit 5
// only when a is.
unsigned sweep_digits(const DOp &d) {
    return d.kind == DOP_U1 ? 1u << d.a : (1u << d.a) | (1u << d.b);
}

// Workgroup barriers between consecutive LDS ops of a pass if the waves of a
// 256-thread sweep split the tile by digit D: one is skipped only between
// two ops that both avoid D.
int split_barriers(const std::vector<DOp> &ops, int D) {
    int count = 0;
    bool have_prev = false, prev_avoids = false;
    for (size_t i = 0; i < ops.size();) {
        const DOp &d = ops[i];
        if (d.kind == DOP_SEG) {
            ++i;
            continue;
        }
        const bool avoids = !((sweep_digits(d) >> D) & 1u);
        if (have_prev && !(prev_avoids && avoids)) ++count;
        have_prev = true;
        prev_avoids = avoids;
        i += d.kind == DOP_GROUP ? 1 + d.ngates : 1;
    }
    return count;
}

// 6-digit tiles: the kernels that sweep them with 256 threads give each wave
// the quarter of the tile whose digit 5 is the wave's index and skip the
// workgroup barrier between two consecutive ops that avoid digit 5.  This
// renames the tile digits of the pass so that the digit among 2..5 that
// costs the fewest barriers becomes digit 5 (the digits above it move down
// by one; digits 0 and 1, the two lowest qubits that give the tile its
// 128-byte runs in HBM, keep their places), then marks every op after which
// the barrier can go.
void split_waves(std::vector<DOp> &ops, DensePass &ps) {
    int best = 5, best_count = split_barriers(ops, 5);
    for (int D = 2; D < 5; ++D) {
        const int c = split_barriers(ops, D);
        if (c < best_count) {
            best = D;
            best_count = c;
        }
    }
    if (best != 5) {
        uint8_t to[8];
        for (int d = 0; d < 8; ++d) to[d] = (uint8_t)(d < best ? d : (d == best ? 5 : (d <= 5 ? d - 1 : d)));
        for (size_t i = 0; i < ops.size();) {
            DOp &h = ops[i];
            if (h.kind == DOP_SEG) {
                uint8_t t[3] = {to[h.a], to[h.b], to[h.smask]};
                std::sort(t, t + 3);
                h.a = t[0];
                h.b = t[1];
                h.smask = t[2];
                ++i;
            } else if (h.kind == DOP_GROUP) {
                const uint8_t a = to[h.a], b = to[h.b];
                h.a = std::min(a, b);
                h.b = std::max(a, b);
                for (int j = 1; j <= h.ngates; ++j) {
                    DOp &m = ops[i + j];
                    m.a = to[m.a];
                    if (m.kind == DOP_CX) m.b = to[m.b];
                }
                h.perm = (uint16_t)group_shape(&ops[i + 1], h.ngates, h.a);
                set_shape_maps(h, &ops[i + 1]);
                i += 1 + h.ngates;
            } else {
                h.a = to[h.a];
                if (h.kind == DOP_CX) h.b = to[h.b];
                ++i;
            }
        }
        uint8_t q[8];
        for (int d = 0; d < ps.k; ++d) q[to[d]] = ps.qubit[d];
        for (int d = 0; d < ps.k; ++d) ps.qubit[d] = q[d];
    }
    DOp *prev = nullptr;
    for (size_t i = 0; i < ops.size();) {
        DOp &d = ops[i];
        if (d.kind == DOP_SEG) {
            ++i;
            continue;
        }
        const bool avoids = !((sweep_digits(d) >> 5) & 1u);
        if (prev && avoids && !((sweep_digits(*prev) >> 5) & 1u)) prev->perm |= (uint16_t)kSkipBarrier;
        prev = &d;
        i += d.kind == DOP_GROUP ? 1 + d.ngates : 1;
    }
}

void group_all(DensePlan &P, bool segments) {
    int shift = 0;
    for (DensePass &ps : P.passes) {
        ps.op_begin += shift;
        ps.op_end += shift;
        const std::vector<DOp> in(P.ops.begin() + ps.op_begin, P.ops.begin() + ps.op_end);
        std::vector<DOp> out =
            (segments && !P.resident && ps.k == kSegTileDigits) ? segment_ops(in, ps.k) : group_ops(in, ps.k);
        if (!P.resident && ps.k == 6) split_waves(out, ps);
        P.ops.erase(P.ops.begin() + ps.op_begin, P.ops.begin() + ps.op_end);
        P.ops.insert(P.ops.begin() + ps.op_begin, out.begin(), out.end());
        const int added = (int)out.size() - (int)in.size();
        ps.op_end += added;
        shift += added;
    }
}

}  // namespace

static DensePlan plan_dense_core(const GateList &g, int k, int low, const PlanOptions &o);

DensePlan plan_dense_opts(const GateList &g, int k, int low, const PlanOptions &o) {
    DensePlan P = plan_dense_core(g, k, low, o);
    if (o.group && o.compose && !o.slot) group_all(P, o.segments);
    return P;
}

static DensePlan plan_dense_core(const GateList &g, int k, int low, const PlanOptions &o) {
    DensePlan P;
    const int n = g.n;
    const bool compose = o.compose, reorder = o.reorder;
    P.roff.push_back(0);
    P.k = k;
    P.resident = (k >= n);
    const int64_t gb = o.g_begin, ge = o.g_end < 0 ? g.m : o.g_end;
    const int64_t m = ge - gb;
    // position h in processing order <-> gate index
    auto gate_of = [&](int64_t h) { return o.forward ? gb + h : ge - 1 - h; };
    auto tag = [&](DOp &d, int64_t gi) {
        if (o.slot && g.op[gi] >= 3) {
            d.b = g.op[gi];
            d.reserved = (uint32_t)(*o.slot)[gi];
        }
    };

    if (P.resident) {
        DensePass pass;
        pass.k = n;
        for (int j = 0; j < n && j < 8; ++j) pass.qubit[j] = (uint8_t)j;
        // Composition needs each map's recipe to be contiguous; gates on
        // other wires in between would interleave recipes.  Collect, per op,
        // its gates first, then emit recipes in op order.
        struct Pending { int digit; std::vector<std::pair<uint8_t, int32_t>> gates; };
        std::vector<Pending> pend;
        std::vector<int> open(n, -1);
        std::vector<DOp> ops;
        for (int64_t h = 0; h < m; ++h) {
            const int64_t gi = gate_of(h);
            const uint8_t op = g.op[gi];
            if (op == 2) {
                DOp d{};
                d.kind = DOP_CX;
                d.a = (uint8_t)g.q0[gi];
                d.b = (uint8_t)g.q1[gi];
                d.ngates = 1;
                open[g.q0[gi]] = -1;
                open[g.q1[gi]] = -1;
                ops.push_back(d);
                continue;
            }
            const int q = g.q0[gi];
            const bool rot = op >= 3;
            if (compose && open[q] >= 0 && ops[open[q]].ngates < 255) {
                DOp &d = ops[open[q]];
                d.ngates++;
                d.smask = (uint16_t)smask_compose(gate_smask(op), d.smask);
                if (rot) d.perm = 0;
                pend[d.map].gates.push_back({op, rot ? g.param[gi] : -1});
            } else {
                DOp d{};
                d.kind = DOP_U1;
                d.a = (uint8_t)q;
                d.ngates = 1;
                d.smask = (uint16_t)gate_smask(op);
                d.perm = rot ? 0 : 1;
                d.map = (uint32_t)pend.size();
                tag(d, gi);
                pend.push_back({q, {{op, rot ? g.param[gi] : -1}}});
                open[q] = (int)ops.size();
                ops.push_back(d);
            }
        }
        for (auto &pd : pend) {
            for (auto &e : pd.gates) {
                P.rop.push_back(e.first);
                P.rparam.push_back(e.second);
            }
            P.roff.push_back((int32_t)P.rop.size());
        }
        P.ops = std::move(ops);
        pass.op_begin = 0;
        pass.op_end = (int)P.ops.size();
        pass.ngates = m;
        P.passes.push_back(pass);
        return P;
    }

    // ---- tiled passes
    std::vector<std::vector<int64_t>> wq(n);
    for (int64_t h = 0; h < m; ++h) {
        const int64_t gi = gate_of(h);
        wq[g.q0[gi]].push_back(h);
        if (g.op[gi] == 2) wq[g.q1[gi]].push_back(h);
    }
    std::vector<size_t> head(n, 0);
    auto wires = [&](int64_t h) -> uint32_t {
        const int64_t gi = gate_of(h);
        uint32_t w = 1u << g.q0[gi];
        if (g.op[gi] == 2) w |= 1u << g.q1[gi];
        return w;
    };
    auto ready = [&](int64_t h) {
        uint32_t w = wires(h);
        for (int q = 0; q < n; ++q)
            if ((w >> q) & 1u)
                if (head[q] >= wq[q].size() || wq[q][head[q]] != h) return false;
        return true;
    };
    const uint32_t lowmask = low >= 32 ? 0xffffffffu : ((1u << std::min(low, n)) - 1u);
    // Schedules, on the head positions hd, every gate whose wires lie in S2
    // and that is next on all of them, until none is; returns their number.
    auto absorb = [&](uint32_t S2, std::vector<size_t> &hd) -> int64_t {
        auto next_on_all = [&](int64_t x) {
            const uint32_t w = wires(x);
            for (int r = 0; r < n; ++r)
                if (((w >> r) & 1u) && (hd[r] >= wq[r].size() || wq[r][hd[r]] != x)) return false;
            return true;
        };
        int64_t got = 0;
        for (bool prog = true; prog;) {
            prog = false;
            for (int r = 0; r < n; ++r) {
                if (!((S2 >> r) & 1u)) continue;
                while (hd[r] < wq[r].size()) {
                    const int64_t x = wq[r][hd[r]];
                    const uint32_t w = wires(x);
                    if ((w & ~S2) || !next_on_all(x)) break;
                    for (int t = 0; t < n; ++t)
                        if ((w >> t) & 1u) hd[t]++;
                    ++got;
                    prog = true;
                }
            }
        }
        return got;
    };
    // Gates a pass would take if its qubit set started as S0 and were then
    // completed to k qubits greedily, each step adding the wires of the
    // ready gate after which the most gates become schedulable.
    auto rollout = [&](uint32_t S0) -> int64_t {
        std::vector<size_t> hd(head), h2;
        uint32_t S2 = S0;
        int64_t total = absorb(S2, hd);
        while (__builtin_popcount(S2) < k) {
            int64_t bg = -1;
            uint32_t bw = 0;
            for (int q = 0; q < n; ++q) {
                if (hd[q] >= wq[q].size()) continue;
                const int64_t x = wq[q][hd[q]];
                const uint32_t w = wires(x);
                bool nxt = true;
                for (int t = 0; t < n; ++t)
                    if (((w >> t) & 1u) && (hd[t] >= wq[t].size() || wq[t][hd[t]] != x)) nxt = false;
                if (!nxt || __builtin_popcount(S2 | w) > k) continue;
                h2 = hd;
                const int64_t gg = absorb(S2 | w, h2);
                if (gg > bg) {
                    bg = gg;
                    bw = w;
                }
            }
            if (bg < 0) break;
            S2 |= bw;
            total += absorb(S2, hd);
        }
        return total;
    };
    int64_t remaining = m;
    while (remaining > 0) {
        uint32_t S = lowmask;
        std::vector<int64_t> sched;
        if (!reorder) {
            // keep the Heisenberg gate order: a pass is a maximal run of
            // consecutive gates whose qubits fit in k
            int64_t h = m - remaining;
            while (h < m && __builtin_popcount(S | wires(h)) <= k) {
                S |= wires(h);
                sched.push_back(h++);
                --remaining;
            }
        }
        for (; reorder;) {
            bool progress = true;
            while (progress) {
                progress = false;
                for (int q = 0; q < n; ++q) {
                    if (!((S >> q) & 1u)) continue;
                    while (head[q] < wq[q].size()) {
                        const int64_t h = wq[q][head[q]];
                        const uint32_t w = wires(h);
                        if ((w & ~S) || !ready(h)) break;
                        for (int r = 0; r < n; ++r)
                            if ((w >> r) & 1u) head[r]++;
                        sched.push_back(h);
                        --remaining;
                        progress = true;
                    }
                }
            }
            if (__builtin_popcount(S) >= k) break;
            // grow the tile by the wires of one ready gate: the one whose
            // greedy completion of the tile schedules the most gates
            // (earliest on ties); without lookahead simply the earliest.
            // Looking only one gate ahead packed 7 % fewer gates per pass
            // into the 6-qubit tiles of random circuits.
            int64_t best = -1, best_gain = -1;
            for (int q = 0; q < n; ++q) {
                if (head[q] >= wq[q].size()) continue;
                const int64_t h = wq[q][head[q]];
                if (!ready(h)) continue;
                if (__builtin_popcount(S | wires(h)) > k) continue;
                const int64_t gain = o.lookahead ? rollout(S | wires(h)) : 0;
                if (gain > best_gain || (gain == best_gain && h < best)) {
                    best = h;
                    best_gain = gain;
                }
            }
            if (best < 0) break;
            S |= wires(best);
        }
        if (sched.empty()) break;  // cannot happen for k >= low + 2
        // pad the qubit set to exactly k qubits with the lowest unused ones
        for (int q = 0; q < n && __builtin_popcount(S) < k; ++q) S |= 1u << q;
        DensePass pass;
        pass.k = k;
        int local[32];
        int j = 0;
        for (int q = 0; q < n; ++q)
            if ((S >> q) & 1u) {
                pass.qubit[j] = (uint8_t)q;
                local[q] = j++;
            }
        pass.op_begin = (int)P.ops.size();
        // per-pass composition with contiguous recipes (see resident case)
        struct Pending { std::vector<std::pair<uint8_t, int32_t>> gates; };
        std::vector<Pending> pend;
        std::vector<int> open(k, -1);
        const int map_base = P.nmaps();
        for (int64_t h : sched) {
            const int64_t gi = gate_of(h);
            const uint8_t op = g.op[gi];
            if (op == 2) {
                DOp d{};
                d.kind = DOP_CX;
                d.a = (uint8_t)local[g.q0[gi]];
                d.b = (uint8_t)local[g.q1[gi]];
                d.ngates = 1;
                open[d.a] = -1;
                open[d.b] = -1;
                P.ops.push_back(d);
                continue;
            }
            const int dg = local[g.q0[gi]];
            const bool rot = op >= 3;
            if (compose && open[dg] >= 0 && P.ops[open[dg]].ngates < 255) {
                DOp &d = P.ops[open[dg]];
                d.ngates++;
                d.smask = (uint16_t)smask_compose(gate_smask(op), d.smask);
                if (rot) d.perm = 0;
                pend[d.map - map_base].gates.push_back({op, rot ? g.param[gi] : -1});
            } else {
                DOp d{};
                d.kind = DOP_U1;
                d.a = (uint8_t)dg;
                d.ngates = 1;
                d.smask = (uint16_t)gate_smask(op);
                d.perm = rot ? 0 : 1;
                d.map = (uint32_t)(map_base + pend.size());
                tag(d, gi);
                pend.push_back({{{op, rot ? g.param[gi] : -1}}});
                open[dg] = (int)P.ops.size();
                P.ops.push_back(d);
            }
        }
        for (auto &pd : pend) {
            for (auto &e : pd.gates) {
                P.rop.push_back(e.first);
                P.rparam.push_back(e.second);
            }
            P.roff.push_back((int32_t)P.rop.size());
        }
        pass.op_end = (int)P.ops.size();
        pass.ngates = (int64_t)sched.size();
        P.passes.push_back(pass);
    }
    return P;
}

std::string plan_check(const DensePlan &P, int n) {
    int expect = 0;
    for (size_t p = 0; p < P.passes.size(); ++p) {
        const DensePass &ps = P.passes[p];
        if (ps.op_begin != expect || ps.op_end < ps.op_begin) return "passes do not tile the op list";
        expect = ps.op_end;
        const int k = ps.k;
        if (k < 1 || k > n || (k < n && k > 8)) return "bad tile size";
        // ascending, except that a 6-digit tile may carry any of its qubits
        // but the two lowest as digit 5
        uint64_t seen = 0;
        for (int j = 0; j < k && j < 8; ++j) {
            if (ps.qubit[j] >= n || ((seen >> ps.qubit[j]) & 1u)) return "tile qubits not distinct";
            seen |= 1ull << ps.qubit[j];
        }
        const int ordered = (!P.resident && k == 6) ? 5 : k;
        for (int j = 1; j < ordered && j < 8; ++j)
            if (ps.qubit[j] <= ps.qubit[j - 1]) return "tile qubits not ascending";
        if (ordered < k && ps.qubit[5] < ps.qubit[1]) return "a lowest qubit moved to digit 5";
        const bool segmented = ps.op_begin < ps.op_end && P.ops[ps.op_begin].kind == DOP_SEG;
        if (segmented && (P.resident || k != kSegTileDigits)) return "SEG header outside a register-tile pass";
        int seg_end = ps.op_begin;
        unsigned triple = 0;
        for (int i = ps.op_begin; i < ps.op_end; ++i) {
            const DOp &d = P.ops[i];
            if (d.kind == DOP_SEG) {
                if (!segmented || i != seg_end) return "SEG header inside a segment";
                if (!(d.a < d.b && d.b < d.smask && d.smask < k) || d.ngates < 1 || i + d.ngates >= ps.op_end)
                    return "bad SEG header";
                triple = (1u << d.a) | (1u << d.b) | (1u << d.smask);
                seg_end = i + 1 + d.ngates;
                continue;
            }
            if (segmented && i >= seg_end) return "op outside every SEG";
            if (segmented) {
                const unsigned dg = d.kind == DOP_CX ? (1u << d.a) | (1u << d.b) : (1u << d.a);
                if (d.kind != DOP_GROUP && (dg & ~triple)) return "op digit outside its SEG triple";
                if (d.kind == DOP_GROUP && i + d.ngates >= seg_end) return "GROUP crosses a SEG boundary";
            }
            if (d.kind == DOP_GROUP) {
                if (d.a == d.b || d.a >= k || d.b >= k || d.ngates < 2 || i + d.ngates >= ps.op_end)
                    return "bad GROUP header";
                for (int j = i + 1; j <= i + d.ngates; ++j) {
                    const DOp &m = P.ops[j];
                    if (m.kind == DOP_GROUP || m.kind == DOP_SEG) return "nested GROUP";
                    if (segmented && (op_digits(m) & ~triple)) return "op digit outside its SEG triple";
                    if (m.a != d.a && m.a != d.b) return "GROUP member outside its pair";
                    if (m.kind == DOP_CX && ((m.b != d.a && m.b != d.b) || m.a == m.b)) return "GROUP CX outside its pair";
                    if (m.kind == DOP_U1 && m.map >= (uint32_t)P.nmaps()) return "map index out of range";
                }
                const unsigned shape = (unsigned)group_shape(&P.ops[(size_t)i + 1], d.ngates, d.a);
                if ((d.perm & ~kSkipBarrier) != shape) return "GROUP shape tag";
                if (shape && (d.map != P.ops[(size_t)i + 2].map ||
                              d.reserved != P.ops[(size_t)i + (d.ngates > 2 ? 3 : 2)].map))
                    return "GROUP shape maps";
                i += d.ngates;
                continue;
            }
            if (d.a >= k || (d.kind == DOP_CX && (d.b >= k || d.a == d.b))) return "op digit outside the tile";
            if (d.kind == DOP_U1 && d.map >= (uint32_t)P.nmaps()) return "map index out of range";
        }
        // a skipped workgroup barrier: only in 6-digit tiled passes, between
        // two ops that both avoid digit 5, so never after a pass's last op
        // (the streaming kernel reads the tile out after that barrier)
        const DOp *prev = nullptr;
        for (int i = ps.op_begin; i < ps.op_end;) {
            const DOp &d = P.ops[i];
            if (d.kind == DOP_SEG) {
                ++i;
                continue;
            }
            if (prev && (prev->perm & kSkipBarrier) && ((sweep_digits(d) >> 5) & 1u))
                return "barrier skipped before an op on digit 5";
            if ((d.perm & kSkipBarrier) && (P.resident || k != 6 || ((sweep_digits(d) >> 5) & 1u)))
                return "barrier skipped after an op on digit 5";
            prev = &d;
            i += d.kind == DOP_GROUP ? 1 + d.ngates : 1;
        }
        if (prev && (prev->perm & kSkipBarrier)) return "barrier skipped after a pass's last op";
    }
    if (expect != (int)P.ops.size()) return "ops outside every pass";
    return "";
}

uint32_t pass_reg_entry(const DensePlan &P, const DensePass &ps) {
    if (ps.op_begin < ps.op_end && P.ops[ps.op_begin].kind == DOP_SEG) {
        const DOp &h = P.ops[ps.op_begin];
        const uint32_t t = (1u << h.a) | (1u << h.b) | (1u << h.smask);
        if (!(t & 3u)) return t;
    }
    return 0x38u;
}

bool plan_segmented(const DensePlan &P) {
    for (const DensePass &ps : P.passes)
        if (!P.resident && ps.k == kSegTileDigits && ps.op_begin < ps.op_end && P.ops[ps.op_begin].kind != DOP_SEG)
            return false;
    return true;
}

void plan_append(DensePlan &all, const DensePlan &part) {
    if (all.roff.empty()) all.roff.push_back(0);
    const int op_off = (int)all.ops.size();
    const uint32_t map_off = (uint32_t)all.nmaps();
    const int32_t rec_off = (int32_t)all.rop.size();
    for (DOp d : part.ops) {
        if (d.kind == DOP_U1) d.map += map_off;
        if (d.kind == DOP_GROUP && (d.perm & ~kSkipBarrier)) {  // a shape's map indices
            d.map += map_off;
            d.reserved += map_off;
        }
        all.ops.push_back(d);
    }
    for (size_t i = 1; i < part.roff.size(); ++i) all.roff.push_back(part.roff[i] + rec_off);
    all.rop.insert(all.rop.end(), part.rop.begin(), part.rop.end());
    all.rparam.insert(all.rparam.end(), part.rparam.begin(), part.rparam.end());
    for (DensePass ps : part.passes) {
        ps.op_begin += op_off;
        ps.op_end += op_off;
        all.passes.push_back(ps);
    }
    all.k = part.k;
    all.resident = part.resident;
}

GradPlan plan_gradient(const GateList &g, int k_heis, int k_fwd, int low, int64_t every) {
    GradPlan G;
    const int64_t m = g.m;
    if (every <= 0) every = m > 0 ? m : 1;
    for (int64_t b = 0; b < m; b += every) G.bounds.push_back(b);
    G.bounds.push_back(m);
    if (G.bounds.size() == 1) G.bounds.push_back(m);  // m == 0: one empty segment
    std::vector<int32_t> slot(m, -1);
    int32_t ns = 0;
    const size_t S = G.bounds.size() - 1;
    for (size_t s = 0; s < S; ++s) {
        G.seg_slot_begin.push_back(ns);
        for (int64_t gi = G.bounds[s]; gi < G.bounds[s + 1]; ++gi)
            if (g.op[gi] >= 3) {
                slot[gi] = ns++;
                G.slot_param.push_back(g.param[gi]);
            }
    }
    G.seg_slot_begin.push_back(ns);
    G.heis.roff.push_back(0);
    G.fwd.roff.push_back(0);
    for (size_t s = 0; s < S; ++s) {
        PlanOptions h;
        h.g_begin = G.bounds[s];
        h.g_end = G.bounds[s + 1];
        G.heis_pass_begin.push_back((int)G.heis.passes.size());
        plan_append(G.heis, plan_dense_opts(g, k_heis, low, h));
        PlanOptions f;
        f.compose = false;
        f.forward = true;
        f.g_begin = G.bounds[s];
        f.g_end = G.bounds[s + 1];
        f.slot = &slot;
        G.fwd_pass_begin.push_back((int)G.fwd.passes.size());
        plan_append(G.fwd, plan_dense_opts(g, k_fwd, low, f));
    }
    G.heis_pass_begin.push_back((int)G.heis.passes.size());
    G.fwd_pass_begin.push_back((int)G.fwd.passes.size());
    return G;
}

SparsePlan plan_sparse(const GateList &g) {
    SparsePlan P;
    const int64_t m = g.m;
    SparsePassDesc cur{};
    cur.g_begin = 0;
    cur.rot_op = -1;
    int ng = 0;
    for (int64_t h = 0; h < m; ++h) {
        const int64_t gi = m - 1 - h;
        const uint8_t op = g.op[gi];
        if (op <= 2) {
            const uint32_t b = op == 2 ? (uint32_t)g.q1[gi] : 0u;
            P.codes.push_back((uint32_t)op | ((uint32_t)g.q0[gi] << 8) | (b << 16));
            ++ng;
            continue;
        }
        cur.g_end = (int32_t)P.codes.size();
        cur.rot_op = op;
        cur.rot_q = g.q0[gi];
        cur.rot_param = g.param[gi];
        cur.ngates = ng + 1;
        P.passes.push_back(cur);
        cur = SparsePassDesc{};
        cur.g_begin = (int32_t)P.codes.size();
        cur.rot_op = -1;
        ng = 0;
    }
    if (ng > 0) {
        cur.g_end = (int32_t)P.codes.size();
        cur.rot_op = -1;
        cur.rot_q = 0;
        cur.rot_param = 0;
        cur.ngates = ng;
        P.passes.push_back(cur);
    }
    return P;
}

// ------------------------------------------------------------ Clifford frame
namespace {

// i^r X^x Z^z (Pauli operators in product form; r mod 4)
struct RawPauli {
    uint64_t x, z;
    int r;
};

RawPauli raw_mul(const RawPauli &A, const RawPauli &B) {
    // X^x1 Z^z1 X^x2 Z^z2 = (-1)^|z1 & x2| X^(x1^x2) Z^(z1^z2)
    return RawPauli{A.x ^ B.x, A.z ^ B.z, (A.r + B.r + 2 * __builtin_popcountll(A.z & B.x)) & 3};
}

// Heisenberg image of a Pauli string's bits under one Clifford code (signs
// not needed here): H swaps x_q and z_q, S^dag . S adds x_q to z_q,
// CX(a -> b) adds x_a to x_b and z_b to z_a.
void heis_bits(uint64_t &x, uint64_t &z, uint32_t code) {
    const int op = code & 0xff, a = (code >> 8) & 0xff, b = (code >> 16) & 0xff;
    const uint64_t xa = (x >> a) & 1ull, za = (z >> a) & 1ull;
    if (op == 0) {
        const uint64_t f = (xa ^ za) << a;
        x ^= f;
        z ^= f;
    } else if (op == 1) {
        z ^= xa << a;
    } else {
        x ^= xa << b;
        z ^= ((z >> b) & 1ull) << a;
    }
}

}  // namespace

FramePlan plan_frame(const GateList &g, const SparsePlan &sp) {
    const int n = g.n;
    FramePlan F;
    // rows of D: DX[j] = D X_j D^dag, DZ[j] = D Z_j D^dag; D starts as the
    // identity and becomes D g for every Clifford g processed
    std::vector<RawPauli> DX(n), DZ(n);
    for (int j = 0; j < n; ++j) {
        DX[j] = RawPauli{1ull << j, 0, 0};
        DZ[j] = RawPauli{0, 1ull << j, 0};
    }
    for (const SparsePassDesc &p : sp.passes) {
        for (int i = p.g_begin; i < p.g_end; ++i) {
            // D g G g^dag D^dag for the generators G that g moves:
            // H: X <-> Z; S: X -> iXZ; CX(c -> t): X_c -> X_c X_t, Z_t -> Z_c Z_t
            const uint32_t code = sp.codes[(size_t)i];
            const int op = code & 0xff, a = (code >> 8) & 0xff, b = (code >> 16) & 0xff;
            if (op == 0) {
                std::swap(DX[a], DZ[a]);
            } else if (op == 1) {
                RawPauli y = raw_mul(DX[a], DZ[a]);
                y.r = (y.r + 1) & 3;
                DX[a] = y;
            } else {
                DX[a] = raw_mul(DX[a], DX[b]);
                DZ[b] = raw_mul(DZ[a], DZ[b]);
            }
        }
        FramePassDesc d{};
        d.ngates = p.ngates;
        d.rot_param = -1;
        if (p.rot_op >= 3) {
            RawPauli P;
            if (p.rot_op == 3) {
                P = DX[p.rot_q];
            } else if (p.rot_op == 5) {
                P = DZ[p.rot_q];
            } else {  // Y = i X Z
                P = raw_mul(DX[p.rot_q], DZ[p.rot_q]);
                P.r = (P.r + 1) & 3;
            }
            // P = i^r X^x Z^z = i^(r - |x & z|) (Hermitian Pauli of x, z);
            // the factor is +-1 because P is Hermitian
            const int a = __builtin_popcountll(P.x & P.z) & 3;
            const int e = (P.r - a) & 3;
            d.pmask = (P.z << n) | P.x;
            d.sign = e == 0 ? 1 : -1;
            d.a = a;
            d.rot_param = p.rot_param;
        }
        F.passes.push_back(d);
    }
    // x part of the actual string D^dag S D of a stored key, bit by bit: the
    // map is linear in the key bits, so column b is the image of the b-th
    // generator (x_b for b < n, z_(b-n) above) under every code in order
    std::vector<uint64_t> colx((size_t)2 * n);
    for (int b = 0; b < 2 * n; ++b) {
        uint64_t x = b < n ? 1ull << b : 0, z = b < n ? 0 : 1ull << (b - n);
        for (uint32_t code : sp.codes) heis_bits(x, z, code);
        colx[(size_t)b] = x;
    }
    F.xrows.assign((size_t)n, 0);
    for (int j = 0; j < n; ++j)
        for (int b = 0; b < 2 * n; ++b)
            if ((colx[(size_t)b] >> j) & 1ull) F.xrows[(size_t)j] |= 1ull << b;
    return F;
}

}  // namespace pp
