// ig_ooo.hip -- the out-of-order engine of Sec. 4.1, simulated on the device
// over finished instruction graphs (the rules are stated with the ig_ooo_*
// declarations in ig.h).
//
// One workgroup simulates one graph, reading the context's records where
// they lie in HBM.  Preparation runs grid-wide: per instruction its lane
// class, duration and number of dependencies (edges are stored sorted by
// target, so the dependency list starts at a lower bound), and the
// successor lists (counted, scanned, filled).  The engine itself is
// sequential in time but parallel inside each round:
//   * the window's state lives in LDS as bitmaps over a ring of
//     IG_OOO_MAX_WINDOW slots (slot = id mod ring): "assignable at the start
//     of the next round" and "assigned";
//   * each instruction's dependency state (how many are unassigned, how many
//     incomplete on foreign lanes, and the count and lane sums of those on
//     its own class's lanes) is kept current in HBM by atomic additions when
//     a dependency is assigned or completes;
//   * after a round (or a completion), only the successors of what changed
//     and the ids that entered the window are evaluated, one thread per
//     successor -- an instruction none of whose dependencies changed cannot
//     have become assignable, so this equals re-evaluating the whole window;
//   * the round's instructions are assigned in id order by one thread per
//     lane class (classes share no lane), walking the ring bitmap's
//     non-empty words;
//   * each lane is a FIFO of in-flight instructions (a linked list through
//     the workspace); with positive durations their ends strictly increase
//     along a lane, so the next completion is the minimum over lane heads
//     and at most one instruction per lane completes at a moment.
#define IG_KERNEL_TU 1
#include "ig_dev.h"

// Per-phase clock totals of the engine's first thread, printed at the end
// (profiling builds only, -DOOO_PROF).
#ifdef OOO_PROF
#include <cstdio>
#define OOO_PROF_DECL u64 prof_t[6] = {0, 0, 0, 0, 0, 0}, prof_last = wall_clock64()
#define OOO_PROF_MARK(k)                    \
    do {                                    \
        const u64 now_ = wall_clock64();    \
        prof_t[k] += now_ - prof_last;      \
        prof_last = now_;                   \
    } while (0)
#define OOO_PROF_REPORT                                                                                         \
    printf("ooo prof n=%u: wait %llu assign %llu prop %llu | wait %llu min+pop %llu prop %llu (wall ticks)\n", n, \
           prof_t[0], prof_t[1], prof_t[2], prof_t[3], prof_t[4], prof_t[5])
#else
#define OOO_PROF_DECL (void)0
#define OOO_PROF_MARK(k) (void)0
#define OOO_PROF_REPORT (void)0
#endif

namespace igd {

constexpr u32 OOO_WR = IG_OOO_MAX_WINDOW;  // ring slots, a power of two
constexpr u32 OOO_WORDS = OOO_WR / 64;     // 64: one summary word covers the ring
constexpr u32 OOO_MAXL = IG_OOO_MAX_LANES;
constexpr u64 OOO_INF = ~0ull;
constexpr u32 OOO_LANE_SHIFT = 11;         // e_cls: class (11 bits) | eager lane + 1
static_assert(OOO_MAXL < 2048, "classes fit the packed class word");
static_assert(OOO_WORDS == 64, "the take summary is one 64-bit word");

// An in-order lane: when it frees up, and its FIFO of in-flight
// instructions (head, tail; linked through the workspace), read and written
// whole.
struct OooLane {
    u64 busy;
    u64 head_end;
    u32 head, tail;
};

struct OooShared {
    u64 take[2][OOO_WORDS];  // ring bitmaps by loop-iteration parity: assignable at the
                             // start of the round that reads them
    u64 asg[OOO_WORDS];      // ring bitmap: assigned, for ids in [first, first + ring)
    OooLane lane[OOO_MAXL];
    // per taken slot: duration; class | (eager lane + 1) << 11; successor
    // list (offset, length)
    u64 e_dur[OOO_WR];
    u32 e_cls[OOO_WR];
    u32 e_o0[OOO_WR];
    u32 e_deg[OOO_WR];
    // changed instructions whose successors are evaluated next: successor
    // list offset and position in the concatenation of the lists
    u32 d_o0[OOO_WR];
    u32 d_pre[OOO_WR];
    u32 d_lane[OOO_WR];
    // by loop-iteration parity (one is read while the other is prepared):
    u64 take_sum[2];   // non-empty words of take[]
    u64 tmin[2];       // the next completion
    u64 cnt[2];        // changed entries << 32 | their successors in total
    u32 firstp[2];     // the first unassigned id
    u64 t;
    u32 win_lo, win_hi;
    u64 r_direct, r_eager, r_makespan;
};

// Whole-record global accesses, field by field (a record behind a global
// pointer has no copy operations of its own).
IGD void ooo_put_slot(ig_ooo_slot* p, const ig_ooo_slot& o) {
    auto q = gmem(p);
    q->lane = o.lane;
    q->how = o.how;
    q->issue = o.issue;
    q->start = o.start;
    q->end = o.end;
}
IGD void ooo_put_rec(OooRec* p, const OooRec& v) {
    auto q = gmem(p);
    q->next = v.next;
    q->o0 = v.o0;
    q->deg = v.deg;
    q->pad = v.pad;
    q->next_end = v.next_end;
}
IGD OooRec ooo_get_rec(const OooRec* p) {
    auto q = gmem(p);
    OooRec v;
    v.next = q->next;
    v.o0 = q->o0;
    v.deg = q->deg;
    v.pad = q->pad;
    v.next_end = q->next_end;
    return v;
}

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
        const i64 lo = gmem(g.box)[d * g.box_stride + x], hi = gmem(g.box)[(3 + d) * g.box_stride + x];
        vol *= hi > lo ? (u64)(hi - lo) : 0ull;
    }
    const u32 kind = gmem(g.kind)[x], mem = gmem(g.mem)[x];
    u32 dev = NONE, cls = 0;
    u64 dur = 0;
    bool engine = false;
    if (kind == IG_KERNEL) {
        dev = mem;
        dur = p.kernel_ns + vol * p.kernel_ns_per_kelem / 1024;
    } else if (kind == IG_COPY) {
        dev = mem >= 2 ? mem : NONE;
        dur = p.copy_ns + vol * p.copy_ns_per_kelem / 1024 + ((gmem(g.flags)[x] & IG_F_INTER_NODE) ? p.inter_node_ns : 0);
    } else if (kind == IG_ALLOC) {
        dur = p.alloc_ns;
    } else if (kind == IG_FREE) {
        dur = p.free_ns;
    } else {
        engine = true;
    }
    // lane class: device d (lanes d * Q ..), the host lanes (class
    // `devices`), or the engine itself (class devices + 1)
    if (engine) {
        cls = p.devices + 1;
    } else if (dev != NONE) {
        if (dev < 2 || dev - 2 >= p.devices) {
            ooo_set_status(g, IG_E_INVALID);
            dev = 2;
        }
        cls = dev - 2;
    } else {
        cls = p.devices;
    }
    gmem(g.cls)[x] = cls;
    gmem(g.dur)[x] = dur;
    const u32 k0 = ooo_lower_bound(g.e_to, g.ne, x), k1 = ooo_lower_bound(g.e_to, g.ne, x + 1);
    auto c = gmem(g.cnt) + x;
    c->uf = k1 - k0;
    c->is = 0;
    c->sumsq = 0;
    gmem(g.out_off)[x] = 0;
    ig_ooo_slot s;
    s.lane = NONE;
    s.how = 0;
    s.issue = OOO_INF;
    s.start = 0;
    s.end = OOO_INF;
    ooo_put_slot(g.out + x, s);
}

// The closing entries of the two offset arrays (one thread per graph).
IGD void ooo_prep_tail(const OooGraph& g) {
    gmem(g.out_off)[g.n] = 0;
}

// An edge the engine can use: ids in range, source before target, sorted
// by target.
IGD bool ooo_edge_ok(const OooGraph& g, u32 e) {
    const u32 f = gmem(g.e_from)[e], t = gmem(g.e_to)[e];
    return t < g.n && f < t && (e == 0 || gmem(g.e_to)[e - 1] <= t);
}

// Preparation, one edge: the check and the successor count of its source.
IGD void ooo_prep_edge(const OooGraph& g, u32 e) {
    if (!ooo_edge_ok(g, e)) {
        ooo_set_status(g, IG_E_INVALID);
        return;
    }
    atomicAdd(&g.out_off[gmem(g.e_from)[e]], 1u);
}

// Preparation, one workgroup per graph: exclusive scan of the successor
// counts over [0, n], each thread summing a contiguous segment; the fill
// cursors start at the offsets.
IGD void ooo_scan(const OooGraph& g, u32* part) {
    const u32 tid = ig_tid(), nt = ig_nthreads(), m = g.n + 1;
    const u32 seg = (m + nt - 1) / nt;
    const u32 lo = tid * seg < m ? tid * seg : m, hi = lo + seg < m ? lo + seg : m;
    u32 s = 0;
    for (u32 i = lo; i < hi; ++i) s += gmem(g.out_off)[i];
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
        const u32 v = gmem(g.out_off)[i];
        gmem(g.out_off)[i] = acc;
        if (i < g.n) gmem(g.rec)[i].next = acc;
        acc += v;
    }
}

IGD void ooo_fill_edge(const OooGraph& g, u32 e) {
    if (!ooo_edge_ok(g, e)) return;  // not counted either
    const u32 pos = atomicAdd(&g.rec[gmem(g.e_from)[e]].next, 1u);
    gmem(g.out_adj)[pos] = gmem(g.e_to)[e];
}

// The lanes [lo, hi) of a class (lo == hi: the engine's own).
IGD void ooo_lanes(const ig_ooo_params& p, u32 cls, u32& lo, u32& hi) {
    const u32 host0 = p.devices * p.lanes_per_device;
    if (cls < p.devices) {
        lo = cls * p.lanes_per_device;
        hi = lo + p.lanes_per_device;
    } else if (cls == p.devices) {
        lo = host0;
        hi = host0 + p.host_lanes;
    } else {
        lo = hi = 0;
    }
}

// A dependency of y changed: it was assigned (to `lane`, NONE for the
// engine's own, which complete at once) or it completed on `lane`.
IGD void ooo_update(const OooGraph& g, const ig_ooo_params& p, u32 y, u32 lane, bool completed) {
    OooCnt* c = g.cnt + y;
    constexpr u64 HI = 1ull << 32;
    if (lane == NONE) {
        if (!completed) atomicAdd(&c->uf, 0ull - 1);  // unasg - 1
        return;
    }
    u32 lo, hi;
    ooo_lanes(p, gmem(g.cls)[y], lo, hi);
    if (lane < lo || lane >= hi) {
        atomicAdd(&c->uf, completed ? 0ull - HI : HI - 1);  // foreign - 1, or unasg - 1 and foreign + 1
        return;
    }
    if (!completed) atomicAdd(&c->uf, 0ull - 1);
    const u64 d = 1ull | (u64)lane << 32;  // inc + 1, suml + lane
    atomicAdd(&c->is, completed ? 0ull - d : d);
    const u64 sq = (u64)lane * lane;
    atomicAdd(&c->sumsq, completed ? 0ull - sq : sq);
}

// Is y assignable now (all dependencies complete, or with eager all
// incomplete ones assigned to one lane of y's class)?  If so, mark it for
// the next round with what the assignment and the following propagation
// need.  Called for any id; filters itself.  The dependency state is read
// from the level-2 cache (agent-scope loads), where the updates' atomics
// were performed.
IGD void ooo_eval(const OooGraph& g, OooShared& sh, const ig_ooo_params& p, u32 y, u32 first, u32 win_end, u64* take,
                  u64* tsum) {
    if (y < first || y >= win_end) return;
    const u32 s = y & (OOO_WR - 1);
    if ((sh.asg[s >> 6] >> (s & 63)) & 1ull) return;
    const OooCnt* c = g.cnt + y;
    const u64 uf = ig_load_agent(&c->uf), is = ig_load_agent(&c->is);
    const u64 sumsq = ig_load_agent(&c->sumsq);
    const u32 unasg = (u32)uf, foreign = (u32)(uf >> 32), inc = (u32)is, suml = (u32)(is >> 32);
    const u32 cls = gmem(g.cls)[y];
    const u32 o0 = gmem(g.out_off)[y], o1 = gmem(g.out_off)[y + 1];
    const u64 dur = gmem(g.dur)[y];
    if (unasg || foreign) return;
    u32 L = NONE;
    if (inc) {
        u32 lo, hi;
        ooo_lanes(p, cls, lo, hi);
        if (!p.eager || lo == hi) return;
        // all on one lane: inc * sum of squares == (sum)^2, in 128 bits
        if ((unsigned __int128)inc * sumsq != (unsigned __int128)suml * suml) return;
        L = suml / inc;
    }
    sh.e_cls[s] = cls | (L == NONE ? 0u : (L + 1) << OOO_LANE_SHIFT);
    sh.e_dur[s] = dur;
    sh.e_o0[s] = o0;
    sh.e_deg[s] = o1 - o0;
    const u64 bit = 1ull << (s & 63);
    const u64 old = atomicOr(&take[s >> 6], bit);
    if (!(old & bit)) atomicOr(tsum, 1ull << (s >> 6));
}

// The entry of the changed list holding successor j of the concatenation.
IGD u32 ooo_entry(const OooShared& sh, u32 nd, u32 j) {
    u32 lo = 0, hi = nd;  // the last entry starting at or before j
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (sh.d_pre[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The successors of the changed instructions (cnt: entries << 32 |
// successors; entry i: successor list from d_o0[i], at position d_pre[i] of
// the concatenation, lane d_lane[i]; one thread per successor): first their
// dependency state is updated, then (after a barrier) they are evaluated,
// with the ids newly in the window [win_lo, win_hi); marks go to take /
// tsum.
IGD void ooo_propagate(const OooGraph& g, OooShared& sh, const ig_ooo_params& p, u64 cnt, bool completed, u32 first,
                       u64* take, u64* tsum) {
    const u32 tid = ig_tid(), nt = ig_nthreads();
    const u32 win_end = (u64)first + p.window < g.n ? first + p.window : g.n;
    const u32 nd = (u32)(cnt >> 32), total = (u32)cnt;
    for (u32 j = tid; j < total; j += nt) {
        const u32 i = ooo_entry(sh, nd, j);
        ooo_update(g, p, gmem(g.out_adj)[sh.d_o0[i] + (j - sh.d_pre[i])], sh.d_lane[i], completed);
    }
    ig_barrier_at(__LINE__);
    for (u32 j = tid; j < total; j += nt) {
        const u32 i = ooo_entry(sh, nd, j);
        ooo_eval(g, sh, p, gmem(g.out_adj)[sh.d_o0[i] + (j - sh.d_pre[i])], first, win_end, take, tsum);
    }
    for (u32 y = sh.win_lo + tid; y < sh.win_hi; y += nt) ooo_eval(g, sh, p, y, first, win_end, take, tsum);
}

// The engine, one workgroup per graph.
IGD void ooo_engine(const OooGraph& g, const ig_ooo_params& p, OooShared& sh) {
    const u32 tid = ig_tid(), nt = ig_nthreads();
    const u32 n = g.n, W = p.window;
    const u32 n_lanes = p.devices * p.lanes_per_device + p.host_lanes;
    const u32 n_cls = p.devices + 2;
    for (u32 w = tid; w < OOO_WORDS; w += nt) sh.take[0][w] = sh.take[1][w] = sh.asg[w] = 0;
    for (u32 l = tid; l < OOO_MAXL; l += nt) {
        OooLane z;
        z.busy = 0;
        z.head_end = OOO_INF;
        z.head = z.tail = NONE;
        sh.lane[l] = z;
    }
    if (tid == 0) {
        for (u32 q = 0; q < 2; ++q) {
            sh.take_sum[q] = 0;
            sh.tmin[q] = OOO_INF;
            sh.cnt[q] = 0;
            sh.firstp[q] = 0;
        }
        sh.t = 0;
        sh.win_lo = 0;
        sh.win_hi = W < n ? W : n;
        sh.r_direct = sh.r_eager = sh.r_makespan = 0;
    }
    ig_barrier_at(__LINE__);
    const bool bad = *(volatile i32*)g.status != 0;
    u64 steps = n ? 1 : 0, rounds = 0, direct = 0, n_eager = 0, makespan = 0;
    bool stalled = false;
    OOO_PROF_DECL;
    if (!bad && n) {
        ooo_propagate(g, sh, p, 0, false, 0, sh.take[0], &sh.take_sum[0]);
        ig_barrier_at(__LINE__);
        // Iteration `it` reads the state of parity it & 1 and prepares that
        // of parity (it + 1) & 1, which nobody reads during the iteration.
        for (u32 it = 0;; ++it) {
            const u32 cur = it & 1, nxt = cur ^ 1;
            const u64 summ = sh.take_sum[cur];
            const u32 first0 = sh.firstp[cur];
            if (summ) {
                OOO_PROF_MARK(0);
                const u64 t = sh.t;
                const u32 fs = first0 & (OOO_WR - 1), w0 = fs >> 6, b0 = fs & 63;
                const u64* tk = sh.take[cur];
                // the round: each class's instructions in id order, one
                // thread per class (classes share no lane); ring order from
                // `first`: word w0 from bit b0, the words after it, then
                // word w0 below bit b0
                // the non-empty words in ring order: rotated so that bit i is
                // word w0 + i; word w0 comes again at the end (bits below b0)
                const u64 rot = w0 ? (summ >> w0) | (summ << (OOO_WORDS - w0)) : summ;
                for (u32 c = tid; c < n_cls; c += nt) {
                    u32 lo, hi;
                    ooo_lanes(p, c, lo, hi);
                    u64 rw = rot;
                    bool tail = b0 && (summ >> w0 & 1ull);
                    while (rw || tail) {
                        u32 w;
                        u64 bits;
                        if (rw) {
                            const u32 i = (u32)__builtin_ctzll(rw);
                            rw &= rw - 1;
                            w = (w0 + i) & (OOO_WORDS - 1);
                            bits = tk[w];
                            if (i == 0) bits &= ~0ull << b0;
                        } else {
                            tail = false;
                            w = w0;
                            bits = tk[w] & ((1ull << b0) - 1);
                        }
                        while (bits) {
                            const u32 b = (u32)__builtin_ctzll(bits);
                            bits &= bits - 1;
                            const u32 s = w * 64 + b;
                            const u32 ec = sh.e_cls[s];
                            if ((ec & 0x7FFu) != c) continue;
                            // independent loads first, so that their latencies overlap
                            const u64 dur = sh.e_dur[s];
                            const u32 eo0 = sh.e_o0[s], edeg = sh.e_deg[s];
                            const u32 y = first0 + ((s - fs) & (OOO_WR - 1));
                            const u32 el = ec >> OOO_LANE_SHIFT;
                            ig_ooo_slot o;
                            o.issue = t;
                            if (lo == hi) {
                                o.lane = NONE;
                                o.how = IG_OOO_ENGINE;
                                o.start = o.end = t;
                            } else {
                                u32 L;
                                if (el) {
                                    L = el - 1u;
                                    o.how = IG_OOO_EAGER;
                                    ++n_eager;
                                } else {
                                    // the lane that frees up first, the lowest on ties
                                    L = lo;
                                    u64 bl = OOO_INF;
                                    for (u32 q0 = lo; q0 < hi; q0 += 4) {
                                        u64 bq[4];
#pragma unroll
                                        for (u32 j = 0; j < 4; ++j) bq[j] = q0 + j < hi ? sh.lane[q0 + j].busy : OOO_INF;
#pragma unroll
                                        for (u32 j = 0; j < 4; ++j)
                                            if (bq[j] < bl) {
                                                bl = bq[j];
                                                L = q0 + j;
                                            }
                                    }
                                    o.how = IG_OOO_DIRECT;
                                    ++direct;
                                }
                                OooLane ln = sh.lane[L];
                                o.lane = L;
                                o.start = t > ln.busy ? t : ln.busy;
                                o.end = o.start + dur;
                                ln.busy = o.end;
                                if (ln.head == NONE) {
                                    ln.head = y;
                                    ln.head_end = o.end;
                                } else {
                                    gmem(g.rec)[ln.tail].next = y;
                                    gmem(g.rec)[ln.tail].next_end = o.end;
                                }
                                ln.tail = y;
                                sh.lane[L] = ln;
                                OooRec r;
                                r.next = NONE;
                                r.o0 = eo0;
                                r.deg = edeg;
                                r.pad = 0;
                                r.next_end = OOO_INF;
                                ooo_put_rec(g.rec + y, r);
                            }
                            makespan = o.end > makespan ? o.end : makespan;
                            ooo_put_slot(g.out + y, o);
                            const u64 at = atomicAdd(&sh.cnt[cur], 1ull << 32 | edeg);
                            sh.d_o0[at >> 32] = eo0;
                            sh.d_pre[at >> 32] = (u32)at;
                            sh.d_lane[at >> 32] = o.lane;
                        }
                    }
                }
                if (tid == 0) {
                    // beside the classes: clear the other parity's round
                    // set, mark this round assigned, advance `first`
                    u64 old = sh.take_sum[nxt];
                    while (old) {
                        const u32 w = (u32)__builtin_ctzll(old);
                        old &= old - 1;
                        sh.take[nxt][w] = 0;
                    }
                    sh.take_sum[nxt] = 0;
                    sh.tmin[nxt] = OOO_INF;
                    sh.cnt[nxt] = 0;
                    u64 sw = summ;
                    while (sw) {
                        const u32 w = (u32)__builtin_ctzll(sw);
                        sw &= sw - 1;
                        sh.asg[w] |= tk[w];
                    }
                    ++rounds;
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
                    sh.firstp[nxt] = f;
                    const u64 lo_w = (u64)first0 + W, hi_w = (u64)f + W;
                    sh.win_lo = lo_w < n ? (u32)lo_w : n;
                    sh.win_hi = hi_w < n ? (u32)hi_w : n;
                }
                ig_barrier_at(__LINE__);
                OOO_PROF_MARK(1);
                ooo_propagate(g, sh, p, sh.cnt[cur], false, sh.firstp[nxt], sh.take[nxt], &sh.take_sum[nxt]);
                ig_barrier_at(__LINE__);
                OOO_PROF_MARK(2);
            } else {
                if (first0 >= n) break;
                OOO_PROF_MARK(3);
                // the next completion: the earliest lane head
                u64 m = OOO_INF;
                for (u32 l = tid; l < n_lanes; l += nt) m = sh.lane[l].head_end < m ? sh.lane[l].head_end : m;
                if (m != OOO_INF) atomicMin(&sh.tmin[cur], m);
                if (tid == 0) {
                    u64 old = sh.take_sum[nxt];
                    while (old) {
                        const u32 w = (u32)__builtin_ctzll(old);
                        old &= old - 1;
                        sh.take[nxt][w] = 0;
                    }
                    sh.take_sum[nxt] = 0;
                    sh.tmin[nxt] = OOO_INF;
                    sh.cnt[nxt] = 0;
                    sh.firstp[nxt] = first0;
                    sh.win_lo = sh.win_hi = 0;
                }
                ig_barrier_at(__LINE__);
                const u64 t = sh.tmin[cur];
                if (t == OOO_INF) {  // nothing in flight and nothing assignable
                    stalled = true;
                    break;
                }
                if (tid == 0) {
                    sh.t = t;
                    ++steps;
                }
                // each lane completes at most its head (ends strictly
                // increase along a lane); one 64-bit counter hands out the
                // entry index and the successor-list position together
                for (u32 l = tid; l < n_lanes; l += nt) {
                    if (sh.lane[l].head_end != t) continue;
                    const u32 x = sh.lane[l].head;
                    const OooRec r = ooo_get_rec(g.rec + x);
                    if (x == sh.lane[l].tail) {
                        sh.lane[l].head = NONE;
                        sh.lane[l].head_end = OOO_INF;
                    } else {
                        sh.lane[l].head = r.next;
                        sh.lane[l].head_end = r.next_end;
                    }
                    const u64 at = atomicAdd(&sh.cnt[cur], 1ull << 32 | r.deg);
                    sh.d_o0[at >> 32] = r.o0;
                    sh.d_pre[at >> 32] = (u32)at;
                    sh.d_lane[at >> 32] = l;
                }
                ig_barrier_at(__LINE__);
                OOO_PROF_MARK(4);
                ooo_propagate(g, sh, p, sh.cnt[cur], true, first0, sh.take[nxt], &sh.take_sum[nxt]);
                ig_barrier_at(__LINE__);
                OOO_PROF_MARK(5);
            }
        }
    }
    if (direct) atomicAdd(&sh.r_direct, direct);
    if (n_eager) atomicAdd(&sh.r_eager, n_eager);
    if (makespan) atomicMax(&sh.r_makespan, makespan);
    ig_barrier_at(__LINE__);
    if (tid == 0) {
        if (stalled) ooo_set_status(g, IG_E_INTERNAL);
        ig_ooo_summary s;
        s.makespan = sh.r_makespan;
        s.direct = sh.r_direct;
        s.eager = sh.r_eager;
        s.steps = steps;
        s.rounds = rounds;
        *g.sum = s;
        OOO_PROF_REPORT;
    }
}

}  // namespace igd

#ifndef IG_HOST_SIM
using namespace igd;

// Each kernel copies its graph descriptor (and the parameters) into
// registers first: read through a pointer, the compiler would reload the
// fields after every store it cannot prove does not alias them.
__global__ void __launch_bounds__(256) ig_ooo_prep_nodes(const OooGraph* gs, ig_ooo_params p) {
    const OooGraph g = gs[blockIdx.y];
    if (blockIdx.x == 0 && threadIdx.x == 0) ooo_prep_tail(g);
    for (u32 x = blockIdx.x * blockDim.x + threadIdx.x; x < g.n; x += gridDim.x * blockDim.x) ooo_prep_node(g, p, x);
}

__global__ void __launch_bounds__(256) ig_ooo_prep_edges(const OooGraph* gs) {
    const OooGraph g = gs[blockIdx.y];
    for (u32 e = blockIdx.x * blockDim.x + threadIdx.x; e < g.ne; e += gridDim.x * blockDim.x) ooo_prep_edge(g, e);
}

__global__ void __launch_bounds__(256) ig_ooo_scan(const OooGraph* gs) {
    __shared__ u32 part[256];
    const OooGraph g = gs[blockIdx.x];
    ooo_scan(g, part);
}

__global__ void __launch_bounds__(256) ig_ooo_fill(const OooGraph* gs) {
    const OooGraph g = gs[blockIdx.y];
    for (u32 e = blockIdx.x * blockDim.x + threadIdx.x; e < g.ne; e += gridDim.x * blockDim.x) ooo_fill_edge(g, e);
}

__global__ void __launch_bounds__(256) ig_ooo_engine(const OooGraph* gs, ig_ooo_params p) {
    __shared__ OooShared sh;
    const OooGraph g = gs[blockIdx.x];
    const ig_ooo_params pp = p;
    ooo_engine(g, pp, sh);
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
