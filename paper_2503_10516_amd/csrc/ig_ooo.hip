// ig_ooo.hip -- the out-of-order engine of Sec. 4.1, simulated on the device
// over finished instruction graphs (the rules are stated with the ig_ooo_*
// declarations in ig.h).
//
// One workgroup simulates one graph, reading the context's records where
// they lie in HBM.  Preparation runs grid-wide: per instruction its lane
// class and duration, the start of its dependency list (edges are stored
// sorted by target, so that is a lower bound), and the successor lists
// (counted, scanned, filled).  The engine itself is sequential in time but
// parallel inside each round:
//   * the window's state lives in LDS as bitmaps over a ring of
//     IG_OOO_MAX_WINDOW slots (slot = id mod ring): "assignable at the start
//     of the next round" and "assigned";
//   * after a round (or a completion), only the successors of what changed
//     and the ids that entered the window are evaluated, by all threads in
//     parallel -- an instruction none of whose dependencies changed cannot
//     have become assignable, so this equals re-evaluating the whole window;
//   * one thread then assigns the round's instructions in id order (lane
//     choice and FIFO order are sequential by definition), walking the ring
//     bitmap word by word;
//   * each lane is a FIFO of in-flight instructions (a linked list through
//     the workspace); with positive durations their ends strictly increase
//     along a lane, so the next completion is the minimum over lane heads
//     and at most one instruction per lane completes at a moment.
#include "ig_dev.h"

namespace igd {

constexpr u32 OOO_WR = IG_OOO_MAX_WINDOW;  // ring slots, a power of two
constexpr u32 OOO_WORDS = OOO_WR / 64;     // 64: one summary word covers the ring
constexpr u32 OOO_MAXL = IG_OOO_MAX_LANES;
constexpr u32 OOO_WIDE = 64;               // successor lists longer than this are walked by all threads
constexpr u32 OOO_WIDE_BIT = 0x80000000u;
constexpr u64 OOO_INF = ~0ull;
static_assert(OOO_WORDS == 64, "the take summary is one 64-bit word");

struct OooShared {
    u64 take[OOO_WORDS];  // ring bitmap: assignable at the start of the next round
    u64 asg[OOO_WORDS];   // ring bitmap: assigned, for ids in [first, first + ring)
    u64 busy[OOO_MAXL];   // when each lane frees up
    u64 head_end[OOO_MAXL];
    u32 head[OOO_MAXL], tail[OOO_MAXL];
    u64 e_dur[OOO_WR];    // per taken slot: duration, lane class, eager lane + 1 (0: direct)
    u32 e_cls[OOO_WR];
    u16 e_lane[OOO_WR];
    u32 done[OOO_WR];     // whose successors are evaluated next (OOO_WIDE_BIT: by all threads)
    u64 take_sum[2];      // non-empty words of take[], by loop-iteration parity (the
                          // next iteration's word is filled while this one's is read)
    u64 tmin[2];          // the next completion, by loop-iteration parity
    u64 t;
    u32 n_done, first, win_lo, win_hi;
};

IGD void ooo_set_status(const OooGraph& g, i32 st) { atomicCAS((unsigned*)g.status, 0u, (unsigned)st); }

IGD u32 ooo_lower_bound(const u32* a, u32 n, u32 v) {
    u32 lo = 0, hi = n;
    while (lo < hi) {
        const u32 mid = lo + (hi - lo) / 2;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Preparation, one instruction: class, duration, dependency-list start,
// initial result slot, zeroed successor count.
IGD void ooo_prep_node(const OooGraph& g, const ig_ooo_params& p, u32 x) {
    u64 vol = 1;
    for (u32 d = 0; d < 3; ++d) {
        const i64 lo = g.box[d * g.box_stride + x], hi = g.box[(3 + d) * g.box_stride + x];
        vol *= hi > lo ? (u64)(hi - lo) : 0ull;
    }
    const u32 kind = g.kind[x], mem = g.mem[x];
    u32 dev = NONE, cls = 0;
    u64 dur = 0;
    bool engine = false;
    if (kind == IG_KERNEL) {
        dev = mem;
        dur = p.kernel_ns + vol * p.kernel_ns_per_kelem / 1024;
    } else if (kind == IG_COPY) {
        dev = mem >= 2 ? mem : NONE;
        dur = p.copy_ns + vol * p.copy_ns_per_kelem / 1024 + ((g.flags[x] & IG_F_INTER_NODE) ? p.inter_node_ns : 0);
    } else if (kind == IG_ALLOC) {
        dur = p.alloc_ns;
    } else if (kind == IG_FREE) {
        dur = p.free_ns;
    } else {
        engine = true;
    }
    if (!engine) {
        const u32 host0 = p.devices * p.lanes_per_device;
        if (dev != NONE) {
            if (dev < 2 || dev - 2 >= p.devices) {
                ooo_set_status(g, IG_E_INVALID);
                dev = 2;
            }
            const u32 lo = (dev - 2) * p.lanes_per_device;
            cls = lo | (lo + p.lanes_per_device) << 16;
        } else {
            cls = host0 | (host0 + p.host_lanes) << 16;
        }
    }
    g.cls[x] = cls;
    g.dur[x] = dur;
    g.in_off[x] = ooo_lower_bound(g.e_to, g.ne, x);
    g.out_off[x] = 0;
    ig_ooo_slot s;
    s.lane = NONE;
    s.how = 0;
    s.issue = OOO_INF;
    s.start = 0;
    s.end = OOO_INF;
    g.out[x] = s;
}

// The closing entries of the two offset arrays (one thread per graph).
IGD void ooo_prep_tail(const OooGraph& g) {
    g.in_off[g.n] = g.ne;
    g.out_off[g.n] = 0;
}

// An edge the engine can use: ids in range, source before target, sorted
// by target.
IGD bool ooo_edge_ok(const OooGraph& g, u32 e) {
    const u32 f = g.e_from[e], t = g.e_to[e];
    return t < g.n && f < t && (e == 0 || g.e_to[e - 1] <= t);
}

// Preparation, one edge: the check and the successor count of its source.
IGD void ooo_prep_edge(const OooGraph& g, u32 e) {
    if (!ooo_edge_ok(g, e)) {
        ooo_set_status(g, IG_E_INVALID);
        return;
    }
    atomicAdd(&g.out_off[g.e_from[e]], 1u);
}

// Preparation, one workgroup per graph: exclusive scan of the successor
// counts over [0, n], each thread summing a contiguous segment; the fill
// cursors start at the offsets.
IGD void ooo_scan(const OooGraph& g, u32* part) {
    const u32 tid = ig_tid(), nt = ig_nthreads(), m = g.n + 1;
    const u32 seg = (m + nt - 1) / nt;
    const u32 lo = tid * seg < m ? tid * seg : m, hi = lo + seg < m ? lo + seg : m;
    u32 s = 0;
    for (u32 i = lo; i < hi; ++i) s += g.out_off[i];
    part[tid] = s;
    ig_barrier_at(__LINE__);
    if (tid == 0) {
        u32 acc = 0;
        for (u32 i = 0; i < nt; ++i) {
            const u32 v = part[i];
            part[i] = acc;
            acc += v;
        }
    }
    ig_barrier_at(__LINE__);
    u32 acc = part[tid];
    for (u32 i = lo; i < hi; ++i) {
        const u32 v = g.out_off[i];
        g.out_off[i] = acc;
        if (i < g.n) g.next[i] = acc;
        acc += v;
    }
}

IGD void ooo_fill_edge(const OooGraph& g, u32 e) {
    if (!ooo_edge_ok(g, e)) return;  // not counted either
    const u32 pos = atomicAdd(&g.next[g.e_from[e]], 1u);
    g.out_adj[pos] = g.e_to[e];
}

// Is y assignable at time t (all dependencies complete, or with eager all
// incomplete ones on one lane of y's class)?  If so, mark it for the next
// round (its non-empty word in *tsum).  Called for any id; filters itself.
IGD void ooo_eval(const OooGraph& g, OooShared& sh, u32 eager, u32 y, u64 t, u32 first, u32 win_end, u64* tsum) {
    if (y < first || y >= win_end) return;
    const u32 s = y & (OOO_WR - 1);
    if ((sh.asg[s >> 6] >> (s & 63)) & 1ull) return;
    const u32 cls = g.cls[y];
    const u32 lo = cls & 0xFFFFu, hi = cls >> 16;
    u32 L = NONE;
    for (u32 k = g.in_off[y], ke = g.in_off[y + 1]; k < ke; ++k) {
        const ig_ooo_slot& d = g.out[g.e_from[k]];
        if (d.end <= t) continue;
        // incomplete (or unassigned: lane NONE, end infinite)
        if (!eager || lo == hi) return;
        const u32 l = d.lane;
        if (l < lo || l >= hi || (L != NONE && l != L)) return;
        L = l;
    }
    sh.e_cls[s] = cls;
    sh.e_dur[s] = g.dur[y];
    sh.e_lane[s] = (u16)(L == NONE ? 0u : L + 1);
    const u64 bit = 1ull << (s & 63);
    const u64 old = atomicOr(&sh.take[s >> 6], bit);
    if (!(old & bit)) atomicOr(tsum, 1ull << (s >> 6));
}

// Evaluate the successors of sh.done[0 .. n_done) and the ids newly in the
// window [win_lo, win_hi); what became assignable is marked in take[] and
// *tsum.
IGD void ooo_propagate(const OooGraph& g, OooShared& sh, u32 eager, u32 window, u64* tsum) {
    const u32 tid = ig_tid(), nt = ig_nthreads();
    const u64 t = sh.t;
    const u32 first = sh.first;
    const u32 win_end = (u64)first + window < g.n ? first + window : g.n;
    const u32 nd = sh.n_done;
    for (u32 i = tid; i < nd; i += nt) {
        const u32 x = sh.done[i];
        const u32 o0 = g.out_off[x], o1 = g.out_off[x + 1];
        if (o1 - o0 > OOO_WIDE) {
            sh.done[i] = x | OOO_WIDE_BIT;
            continue;
        }
        for (u32 j = o0; j < o1; ++j) ooo_eval(g, sh, eager, g.out_adj[j], t, first, win_end, tsum);
    }
    for (u32 y = sh.win_lo + tid; y < sh.win_hi; y += nt) ooo_eval(g, sh, eager, y, t, first, win_end, tsum);
    ig_barrier_at(__LINE__);
    for (u32 i = 0; i < nd; ++i) {
        const u32 xw = sh.done[i];
        if (!(xw & OOO_WIDE_BIT)) continue;
        const u32 x = xw & ~OOO_WIDE_BIT;
        const u32 o0 = g.out_off[x], o1 = g.out_off[x + 1];
        for (u32 j = o0 + tid; j < o1; j += nt) ooo_eval(g, sh, eager, g.out_adj[j], t, first, win_end, tsum);
    }
}

// The engine, one workgroup per graph.
IGD void ooo_engine(const OooGraph& g, const ig_ooo_params& p, OooShared& sh) {
    const u32 tid = ig_tid(), nt = ig_nthreads();
    const u32 n = g.n, W = p.window, eager = p.eager;
    const u32 n_lanes = p.devices * p.lanes_per_device + p.host_lanes;
    for (u32 w = tid; w < OOO_WORDS; w += nt) sh.take[w] = sh.asg[w] = 0;
    for (u32 l = tid; l < OOO_MAXL; l += nt) {
        sh.busy[l] = 0;
        sh.head_end[l] = OOO_INF;
        sh.head[l] = sh.tail[l] = NONE;
    }
    if (tid == 0) {
        sh.take_sum[0] = sh.take_sum[1] = 0;
        sh.t = 0;
        sh.first = 0;
        sh.n_done = 0;
        sh.win_lo = 0;
        sh.win_hi = W < n ? W : n;
        sh.tmin[0] = sh.tmin[1] = OOO_INF;
    }
    ig_barrier_at(__LINE__);
    const bool bad = *(volatile i32*)g.status != 0;
    u64 steps = n ? 1 : 0, rounds = 0, direct = 0, n_eager = 0, makespan = 0;
    bool stalled = false;
    if (!bad && n) {
        ooo_propagate(g, sh, eager, W, &sh.take_sum[0]);
        ig_barrier_at(__LINE__);
        for (u32 it = 0;; ++it) {
            // this iteration's round was marked under parity it & 1; the
            // next one is marked under the other parity, which the assigning
            // thread clears before the barrier that precedes the marking
            u64* next_sum = &sh.take_sum[(it + 1) & 1];
            const u64 summ = sh.take_sum[it & 1];
            if (summ) {
                if (tid == 0) {
                    *next_sum = 0;
                    sh.tmin[(it + 1) & 1] = OOO_INF;
                    const u64 t = sh.t;
                    const u32 first0 = sh.first;
                    const u32 fs = first0 & (OOO_WR - 1), w0 = fs >> 6, b0 = fs & 63;
                    u32 nd = 0;
                    // ring order from `first`: word w0 from bit b0, the words
                    // after it, then word w0 below bit b0
                    for (u32 step = 0; step <= OOO_WORDS; ++step) {
                        const u32 w = (w0 + step) & (OOO_WORDS - 1);
                        if (!((summ >> w) & 1ull)) continue;
                        u64 bits = sh.take[w];
                        if (step == 0) bits &= ~0ull << b0;
                        else if (step == OOO_WORDS) bits &= b0 ? (1ull << b0) - 1 : 0ull;
                        sh.take[w] &= ~bits;
                        while (bits) {
                            const u32 b = (u32)__builtin_ctzll(bits);
                            bits &= bits - 1;
                            const u32 s = w * 64 + b;
                            const u32 y = first0 + ((s - fs) & (OOO_WR - 1));
                            const u32 cls = sh.e_cls[s];
                            const u32 lo = cls & 0xFFFFu, hi = cls >> 16;
                            ig_ooo_slot o;
                            o.issue = t;
                            if (lo == hi) {
                                o.lane = NONE;
                                o.how = IG_OOO_ENGINE;
                                o.start = o.end = t;
                            } else {
                                u32 L;
                                if (sh.e_lane[s]) {
                                    L = sh.e_lane[s] - 1u;
                                    o.how = IG_OOO_EAGER;
                                    ++n_eager;
                                } else {
                                    L = lo;
                                    for (u32 q = lo + 1; q < hi; ++q)
                                        if (sh.busy[q] < sh.busy[L]) L = q;
                                    o.how = IG_OOO_DIRECT;
                                    ++direct;
                                }
                                o.lane = L;
                                o.start = t > sh.busy[L] ? t : sh.busy[L];
                                o.end = o.start + sh.e_dur[s];
                                sh.busy[L] = o.end;
                                if (sh.head[L] == NONE) {
                                    sh.head[L] = y;
                                    sh.head_end[L] = o.end;
                                } else {
                                    g.next[sh.tail[L]] = y;
                                }
                                sh.tail[L] = y;
                                g.next[y] = NONE;
                            }
                            makespan = o.end > makespan ? o.end : makespan;
                            g.out[y] = o;
                            sh.asg[s >> 6] |= 1ull << (s & 63);
                            sh.done[nd++] = y;
                        }
                    }
                    ++rounds;
                    // advance the first unassigned id over the assigned run
                    u32 f = first0;
                    while (f < n) {
                        const u32 s = f & (OOO_WR - 1), w = s >> 6, b = s & 63;
                        const u64 run = ~(sh.asg[w] >> b);  // zero bits: assigned, from slot s on
                        u32 adv = run ? (u32)__builtin_ctzll(run) : 64u;
                        if (adv > 64 - b) adv = 64 - b;
                        if (adv > n - f) adv = n - f;
                        if (adv == 0) break;
                        const u64 m = adv == 64 ? ~0ull : ((1ull << adv) - 1) << b;
                        sh.asg[w] &= ~m;
                        f += adv;
                        if (adv < 64 - b) break;
                    }
                    sh.first = f;
                    const u64 lo_w = (u64)first0 + W, hi_w = (u64)f + W;
                    sh.win_lo = lo_w < n ? (u32)lo_w : n;
                    sh.win_hi = hi_w < n ? (u32)hi_w : n;
                    sh.n_done = nd;
                }
                ig_barrier_at(__LINE__);
                ooo_propagate(g, sh, eager, W, next_sum);
                ig_barrier_at(__LINE__);
            } else {
                if (sh.first >= n) break;
                // the next completion: the earliest lane head
                u64 m = OOO_INF;
                for (u32 l = tid; l < n_lanes; l += nt) m = sh.head_end[l] < m ? sh.head_end[l] : m;
                if (m != OOO_INF) atomicMin(&sh.tmin[it & 1], m);
                if (tid == 0) {
                    *next_sum = 0;
                    sh.tmin[(it + 1) & 1] = OOO_INF;
                    sh.n_done = 0;
                    sh.win_lo = sh.win_hi = 0;
                }
                ig_barrier_at(__LINE__);
                const u64 t = sh.tmin[it & 1];
                if (t == OOO_INF) {  // nothing in flight and nothing assignable
                    stalled = true;
                    break;
                }
                if (tid == 0) {
                    sh.t = t;
                    ++steps;
                }
                for (u32 l = tid; l < n_lanes; l += nt) {
                    if (sh.head_end[l] != t) continue;
                    const u32 x = sh.head[l];
                    if (x == sh.tail[l]) {
                        sh.head[l] = NONE;
                        sh.head_end[l] = OOO_INF;
                    } else {
                        const u32 nx = g.next[x];
                        sh.head[l] = nx;
                        sh.head_end[l] = g.out[nx].end;
                    }
                    sh.done[atomicAdd(&sh.n_done, 1u)] = x;
                }
                ig_barrier_at(__LINE__);
                ooo_propagate(g, sh, eager, W, next_sum);
                ig_barrier_at(__LINE__);
            }
        }
    }
    if (tid == 0) {
        if (stalled) ooo_set_status(g, IG_E_INTERNAL);
        ig_ooo_summary s;
        s.makespan = makespan;
        s.direct = direct;
        s.eager = n_eager;
        s.steps = steps;
        s.rounds = rounds;
        *g.sum = s;
    }
}

}  // namespace igd

#ifndef IG_HOST_SIM
using namespace igd;

__global__ void __launch_bounds__(256) ig_ooo_prep_nodes(const OooGraph* gs, ig_ooo_params p) {
    const OooGraph& g = gs[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) ooo_prep_tail(g);
    for (u32 x = blockIdx.x * blockDim.x + threadIdx.x; x < g.n; x += gridDim.x * blockDim.x) ooo_prep_node(g, p, x);
}

__global__ void __launch_bounds__(256) ig_ooo_prep_edges(const OooGraph* gs) {
    const OooGraph& g = gs[blockIdx.y];
    for (u32 e = blockIdx.x * blockDim.x + threadIdx.x; e < g.ne; e += gridDim.x * blockDim.x) ooo_prep_edge(g, e);
}

__global__ void __launch_bounds__(256) ig_ooo_scan(const OooGraph* gs) {
    __shared__ u32 part[256];
    ooo_scan(gs[blockIdx.x], part);
}

__global__ void __launch_bounds__(256) ig_ooo_fill(const OooGraph* gs) {
    const OooGraph& g = gs[blockIdx.y];
    for (u32 e = blockIdx.x * blockDim.x + threadIdx.x; e < g.ne; e += gridDim.x * blockDim.x) ooo_fill_edge(g, e);
}

__global__ void __launch_bounds__(256) ig_ooo_engine(const OooGraph* gs, ig_ooo_params p) {
    __shared__ OooShared sh;
    ooo_engine(gs[blockIdx.x], p, sh);
}

namespace igrt {
// Preparation grids: enough workgroups per graph to cover the largest one,
// capped; every kernel strides.
int launch_ooo(const igd::OooGraph* d_graphs, unsigned n_graphs, uint64_t max_n, uint64_t max_ne,
               const ig_ooo_params* p, void* stream) {
    if (!n_graphs) return 0;
    hipStream_t st = (hipStream_t)stream;
    auto blocks = [](uint64_t m) {
        uint64_t b = (m + 255) / 256;
        return (unsigned)(b < 1 ? 1 : b > 1024 ? 1024 : b);
    };
    hipLaunchKernelGGL(ig_ooo_prep_nodes, dim3(blocks(max_n), n_graphs), dim3(256), 0, st, d_graphs, *p);
    hipLaunchKernelGGL(ig_ooo_prep_edges, dim3(blocks(max_ne), n_graphs), dim3(256), 0, st, d_graphs);
    hipLaunchKernelGGL(ig_ooo_scan, dim3(n_graphs), dim3(256), 0, st, d_graphs);
    hipLaunchKernelGGL(ig_ooo_fill, dim3(blocks(max_ne), n_graphs), dim3(256), 0, st, d_graphs);
    hipLaunchKernelGGL(ig_ooo_engine, dim3(n_graphs), dim3(256), 0, st, d_graphs, *p);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
}  // namespace igrt
#endif
