// ig_kernels.hip -- instruction-graph generation on gfx950.
//
// One workgroup analyses one stream (context); a launch may cover many
// streams (one workgroup each).  Within a workgroup the control flow is
// uniform: every thread walks the same command sequence, and the parallel
// parts of each step are spread over the threads:
//   * chunk split, range mappers, cell lookup, debug checks: over
//     (chunk, access) pairs;
//   * allocation phase, coherence copies, kernels, reader updates: over
//     simulated memories -- the thread owning a memory does every update of
//     that memory's allocation maps (no atomics needed there);
//   * id/offset assignment: block-wide exclusive scans in LDS;
//   * edge output: each instruction's sources are sorted, de-duplicated with
//     their kinds OR-ed, staged, then written in (to, from) order after a
//     scan of the per-instruction counts.
// Paper passages: Sec. 3.1 (split), 3.2 (allocation), 3.3 (coherence),
// 3.5 (horizons/epochs), Table 1 (instruction kinds), the dependency-kind
// legend of the IDAG figure (Sec. 3.6), Sec. 4.1 (topological emission),
// Sec. 4.3 (lookahead), Sec. 4.4 (debug checks).
#include <mutex>

#define IG_KERNEL_TU 1
#include "ig_dev.h"

namespace igd {

// ===========================================================================
// Workgroup-shared scratch (LDS)
// ===========================================================================
struct Shared {
    Scalars s;
    u32 scan[MAX_THREADS / 64];
    u32 scan_tmp[16];
    u32 total;
    u32 flag;        // generic OR flag
    u32 flag2;
    u32 unit_first;  // first instruction id of the command being compiled
    u32 unit_n;      // instructions of that command so far
    u32 stage_top;   // staged edges of that command
    u32 copy_top;    // coherence copies found for that task
    u32 nfree;       // allocations freed in the allocation phase
    u32 t_dims, t_nacc, t_id, t_cmd;
    u32 t_stamps;  // some write may leave its chunk's dim-0 range: check overlaps cell by cell
    u64 t_wbufs;   // buffers the task writes (bit per buffer)
    u32 t_par;     // kernels may be emitted in parallel (see kernels_emit_par)
    u32 t_gmask;   // with t_par: accesses read through one shared source list per device
    i64 t_lo[3], t_hi[3];
    u32 n_alloc_instr, n_new_allocs, n_copies, n_kernels;
    u32 win_first, win_n;  // lookahead window (queue positions)
    u32 t_covered;         // every requirement of the current task lies in a live allocation
    u32 do_horizon;
    u32 miss_total;
    u64 tick;
    u64 wkey[256 * 16];  // per-worker stale-cell keys of one consumer (small case)
    u32 wval[256 * 16];
    u32 rbs_head[MAX_THREADS];  // per thread: a private run of free reader blocks (0: none)
    u16 rbs_mem[MAX_THREADS];   // ... of this memory
};

IGD u32 tid() { return ig_tid(); }
IGD u32 nt() { return ig_nthreads(); }
#define bar() ig_barrier_at(__LINE__)

IGD void set_error(Shared& sh, i32 code) { atomicCAS((u32*)&sh.s.error, 0u, (u32)code); }
// a capacity overflow, with the capacity that ran out (first one wins)
IGD void cap_error(Shared& sh, u32 what) {
    if (atomicCAS((u32*)&sh.s.error, 0u, (u32)IG_E_CAPACITY) == 0u) sh.s.cap_what = what;
}

// Uniform read of the error flag: every thread sees the same value because
// nobody can set it between the two barriers.
IGD bool failed(Shared& sh) {
    bar();
    const bool e = sh.s.error != 0;
    bar();
    return e;
}

// Phase profile (IG_PHASE_PROFILE builds): device-clock ticks spent since the
// previous checkpoint are charged to phase `id`.
enum Phase : u32 {
    PH_INTAKE_REGIONS, PH_INTAKE_CHECKS, PH_LOOKAHEAD, PH_COMPILE_REGIONS, PH_ALLOC, PH_COH_COUNT, PH_SCANS,
    PH_COH_EMIT, PH_INBOX, PH_KERNELS, PH_EDGES_OUT, PH_SYNC, PH_OTHER, PH_N
};
IGD void tick(DevCtx& c, Shared& sh, u32 id) {
#ifdef IG_PHASE_PROFILE
    if (tid() == 0) {
        const u64 now = ig_clock();
        c.phase[id] += now - sh.tick;
        c.phase[16 + id] += 1;
        sh.tick = now;
    }
#else
    (void)c;
    (void)sh;
    (void)id;
#endif
}

// Uniform read of a word that threads may have just written (first barrier)
// and that one thread may change right after (second barrier).
IGD u32 uniform(const u32& v) {
    bar();
    const u32 x = v;
    bar();
    return x;
}

// ===========================================================================
// Scans: inclusive scan inside each 64-lane wave with shuffles, wave totals
// through LDS (one barrier).  The workgroup size is a multiple of 64.
// ===========================================================================
IGD u32 wave_incl_scan(u32 v) {
    const u32 lane = tid() & 63;
    for (u32 off = 1; off < 64; off <<= 1) {
        const u32 y = ig_shfl_up(v, off);
        if (lane >= off) v += y;
    }
    return v;
}

// exclusive prefix of per-thread values over the workgroup; *total = sum
IGD u32 block_excl(Shared& sh, u32 v, u32* total) {
    const u32 incl = wave_incl_scan(v);
    const u32 w = tid() >> 6, nw = nt() >> 6;
    if ((tid() & 63) == 63) sh.scan[w] = incl;
    bar();
    u32 base = 0, all = 0;
    for (u32 i = 0; i < nw; ++i) {
        const u32 x = sh.scan[i];
        if (i < w) base += x;
        all += x;
    }
    bar();
    *total = all;
    return base + incl - v;
}

// Block-wide exclusive scan of a u32 array in global memory; returns total.
IGN u32 block_exscan(Shared& sh, u32* a, u32 n) {
    const u32 T = nt(), t = tid();
    const u32 per = (n + T - 1) / T;
    const u32 lo = t * per < n ? t * per : n;
    const u32 hi = lo + per < n ? lo + per : n;
    u32 sum = 0;
    for (u32 i = lo; i < hi; ++i) sum += a[i];
    u32 total;
    u32 run = block_excl(sh, sum, &total);
    for (u32 i = lo; i < hi; ++i) {
        const u32 v = a[i];
        a[i] = run;
        run += v;
    }
    bar();
    return total;
}

// ===========================================================================
// Heap: power-of-two blocks of 32-bit words for grids and map arrays.
// Only thread 0 allocates and frees (between barriers).
// ===========================================================================
IGD u32 heap_alloc(DevCtx& c, Shared& sh, u32 words) {
    u32 need = words + 4, k = 4;
    while ((1u << k) < need) ++k;
    u32 off;
    if (c.heap_free[k]) {
        off = c.heap_free[k];
        c.heap_free[k] = c.heap[off + 2];
    } else {
        if ((u64)sh.s.heap_top + (1ull << k) > c.cap_heap) {
            cap_error(sh, IG_CAP_STATE);
            return 0;
        }
        off = sh.s.heap_top;
        sh.s.heap_top += 1u << k;
    }
    c.heap[off] = k;
    return off + 4;
}

IGD void heap_release(DevCtx& c, u32 p) {
    if (!p) return;
    const u32 off = p - 4, k = c.heap[off];
    c.heap[off + 2] = c.heap_free[k];
    c.heap_free[k] = off;
}

IGD u32* W32(DevCtx& c, u32 off) { return c.heap + off; }
IGD u64* W64(DevCtx& c, u32 off) { return (u64*)(c.heap + off); }
IGD i64* WI64(DevCtx& c, u32 off) { return (i64*)(c.heap + off); }
IGD AmCell* am_cells(DevCtx& c, const DAlloc& a) { return (AmCell*)(c.heap + a.am_off); }

IGD AmCell am_load(const AmCell* p) {
#ifdef IG_HOST_SIM
    return *p;
#else
    const uint4 v = *(const uint4*)p;
    AmCell e;
    e.w = v.x;
    e.r0 = v.y;
    e.r1 = v.z;
    e.ov = v.w;
    return e;
#endif
}


// ===========================================================================
// Reader lists: singly linked blocks of 7 slots; owned by one memory's
// worker.  A slot holds a reader id, or NONE, or -- with RB_RANGE set -- the
// first id of a run of consecutive readers whose length is in the next slot
// of the same block (the kernels of one device reading one region).
// ===========================================================================
constexpr u32 RB_RANGE = 0x80000000u;

// f(first, count) for every reader entry of a list
template <class F>
IGD void rd_each(const DevCtx& c, u32 head, F f) {
    for (u32 h = head; h; h = c.rb[h * 8 + 7])
        for (u32 q = 0; q < RB_SLOTS; ++q) {
            const u32 v = c.rb[h * 8 + q];
            if (v == NONE) continue;
            if (v & RB_RANGE) {
                f(v & ~RB_RANGE, c.rb[h * 8 + q + 1]);
                ++q;
            } else {
                f(v, 1u);
            }
        }
}
// Free lists of reader blocks, one per memory: a 64-bit head (tag << 32 |
// block) changed only by compare-and-swap, the tag counting every change, so
// that threads taking and returning blocks of one memory at once cannot be
// fooled by a head that was taken and returned in between.
// A thread takes up to RB_TAKE blocks of a memory's free list with one
// compare-and-swap and keeps the rest as a private run (rbs_head), used
// before the shared list is touched again; the run goes back to the free
// list when the thread needs another memory's blocks and at the end of
// every compiled command (rb_stash_return).
constexpr u32 RB_TAKE = 4;
IGD void rd_clear(DevCtx& c, u32 m, u32* head);
IGD void rb_stash_return(DevCtx& c, Shared& sh) {
    u32* h = &sh.rbs_head[tid()];
    if (*h) rd_clear(c, sh.rbs_mem[tid()], h);
}
IGN u32 rb_alloc_slow(DevCtx& c, Shared& sh, u32 m);
IGD u32 rb_alloc(DevCtx& c, Shared& sh, u32 m) {
    u32& run = sh.rbs_head[tid()];
    if (run && sh.rbs_mem[tid()] == m) {
        const u32 h = run;
        run = c.rb[h * 8 + 7];
        return h;
    }
    return rb_alloc_slow(c, sh, m);
}
// out of line: the shared free list, or fresh blocks
IGN u32 rb_alloc_slow(DevCtx& c, Shared& sh, u32 m) {
    u32& run = sh.rbs_head[tid()];
    rb_stash_return(c, sh);
    u64 old = atomicAdd(&c.rb_free[m], 0ull);
    while ((u32)old) {
        const u32 h = (u32)old;
        u32 last = h;
        for (u32 k = 1; k < RB_TAKE && c.rb[last * 8 + 7]; ++k) last = c.rb[last * 8 + 7];
        const u64 nw = (((old >> 32) + 1) << 32) | c.rb[last * 8 + 7];
        const u64 seen = atomicCAS(&c.rb_free[m], old, nw);
        if (seen == old) {
            // the tag did not change, so h .. last were still linked: they are ours
            c.rb[last * 8 + 7] = 0;
            run = last == h ? 0u : c.rb[h * 8 + 7];
            sh.rbs_mem[tid()] = (u16)m;
            return h;
        }
        old = seen;
    }
    u32 i = atomicAdd(&sh.s.rb_top, 1u);
    if (i >= c.cap_rb) {
        cap_error(sh, IG_CAP_READERS);
        return 0;
    }
    return i;
}

IGD bool rd_put(DevCtx& c, u32 h, u32 x) {
    u32* blk = c.rb + h * 8;
    for (u32 s = 0; s < RB_SLOTS; ++s)
        if (blk[s] == NONE) {
            blk[s] = x;
            return true;
        }
    return false;
}

IGN void rd_compact(DevCtx& c, Shared& sh, u32 m, u32* head);

// the newest block of a list holds a reader that now reads as S or absent
IGD bool rd_stale_head(const DevCtx& c, const Shared& sh, u32 h) {
    bool stale = false;
    for (u32 q = 0; q < RB_SLOTS; ++q) {
        const u32 v = c.rb[h * 8 + q];
        if (v == NONE) continue;
        stale = stale || (v & ~RB_RANGE) < sh.s.S;
        if (v & RB_RANGE) ++q;
    }
    return stale;
}

IGD void rd_append(DevCtx& c, Shared& sh, u32 m, u32* head, u32 x) {
    u32 h = *head;
    if (h && rd_put(c, h, x)) return;
    if (h && c.rb[h * 8 + 7] && rd_stale_head(c, sh, h)) {
        // a further block is due and even the newest readers have aged:
        // first drop what no longer matters
        rd_compact(c, sh, m, head);
        h = *head;
        if (h && rd_put(c, h, x)) return;
    }
    const u32 n = rb_alloc(c, sh, m);
    if (!n) return;
    u32* blk = c.rb + n * 8;
    blk[0] = x;
    for (u32 s = 1; s < RB_SLOTS; ++s) blk[s] = NONE;
    blk[7] = h;
    *head = n;
}

// Return a list to its memory's free list (the whole chain at once).
IGD void rd_clear(DevCtx& c, u32 m, u32* head) {
    const u32 first = *head;
    if (!first) return;
    u32 last = first;
    while (c.rb[last * 8 + 7]) last = c.rb[last * 8 + 7];
    u64 old = atomicAdd(&c.rb_free[m], 0ull);
    while (true) {
        c.rb[last * 8 + 7] = (u32)old;
        __threadfence_block();
        const u64 seen = atomicCAS(&c.rb_free[m], old, (((old >> 32) + 1) << 32) | first);
        if (seen == old) break;
        old = seen;
    }
    *head = 0;
}

// a run of n >= 2 consecutive readers first..first+n-1
IGD void rd_append_range(DevCtx& c, Shared& sh, u32 m, u32* head, u32 first, u32 n) {
    const u32 h = *head;
    if (h) {
        u32* blk = c.rb + h * 8;
        for (u32 s = 0; s + 1 < RB_SLOTS; ++s)
            if (blk[s] == NONE && blk[s + 1] == NONE) {
                blk[s + 1] = n;
                blk[s] = first | RB_RANGE;
                return;
            }
    }
    const u32 b = rb_alloc(c, sh, m);
    if (!b) return;
    u32* blk = c.rb + b * 8;
    blk[0] = first | RB_RANGE;
    blk[1] = n;
    for (u32 s = 2; s < RB_SLOTS; ++s) blk[s] = NONE;
    blk[7] = h;
    *head = b;
}

IGN u32 rd_copy(DevCtx& c, Shared& sh, u32 m, u32 head) {
    u32 out = 0;
    rd_each(c, head, [&](u32 first, u32 n) {
        if (n == 1)
            rd_append(c, sh, m, &out, first);
        else
            rd_append_range(c, sh, m, &out, first, n);
    });
    return out;
}

// Rewrite a reader list keeping only what still matters: readers before the
// last epoch go, readers before the synchronisation point S all read as S
// and are kept as one entry S (S only grows and stays below later epochs
// exactly when they do, so the substitution is exact for the future too).
IGN void rd_compact(DevCtx& c, Shared& sh, u32 m, u32* head) {
    const u32 S = sh.s.S, E = sh.s.E;
    u32 out = 0;
    bool has_s = false;
    auto put = [&](u32 first, u32 n) {
        if (n == 1) {
            if (!(out && rd_put(c, out, first))) {
                const u32 b = rb_alloc(c, sh, m);
                if (!b) return;
                u32* blk = c.rb + b * 8;
                blk[0] = first;
                for (u32 q = 1; q < RB_SLOTS; ++q) blk[q] = NONE;
                blk[7] = out;
                out = b;
            }
        } else {
            rd_append_range(c, sh, m, &out, first, n);
        }
    };
    rd_each(c, *head, [&](u32 first, u32 n) {
        const u32 end = first + n;
        u32 lo = first < E ? E : first;
        if (lo >= end) return;
        if (lo < S) {
            has_s = true;
            lo = S;
        }
        if (lo < end) put(lo, end - lo);
    });
    if (has_s) put(S, 1);
    rd_clear(c, m, head);
    *head = out;
}

// Lazy horizon/epoch substitution (Sec. 3.5): ids below the synchronisation
// point read as S; readers from before the last epoch no longer exist.
IGD u32 eff_w(const Shared& sh, u32 w) { return w < sh.s.S ? sh.s.S : w; }
IGD bool eff_r(const Shared& sh, u32 r, u32& out) {
    if (r < sh.s.E) return false;
    out = r < sh.s.S ? sh.s.S : r;
    return true;
}

// ===========================================================================
// Per-thread source lists: (id << 8 | kind), sorted and de-duplicated.
// ===========================================================================
IGN void msort64(u64* a, u64* tmp, u32 n) {
    u64* src = a;
    u64* dst = tmp;
    for (u32 w = 1; w < n; w <<= 1) {
        for (u32 i = 0; i < n; i += 2 * w) {
            u32 m = i + w < n ? i + w : n, e = i + 2 * w < n ? i + 2 * w : n;
            u32 p = i, q = m, o = i;
            while (p < m && q < e) dst[o++] = (src[q] < src[p]) ? src[q++] : src[p++];
            while (p < m) dst[o++] = src[p++];
            while (q < e) dst[o++] = src[q++];
        }
        u64* t = src;
        src = dst;
        dst = t;
    }
    if (src != a)
        for (u32 i = 0; i < n; ++i) a[i] = src[i];
}

// stable sort of (key, val) pairs by key
IGN void msort_kv(u64* k, u32* v, u64* k2, u32* v2, u32 n) {
    u64* sk = k;
    u32* sv = v;
    u64* dk = k2;
    u32* dv = v2;
    for (u32 w = 1; w < n; w <<= 1) {
        for (u32 i = 0; i < n; i += 2 * w) {
            u32 m = i + w < n ? i + w : n, e = i + 2 * w < n ? i + 2 * w : n;
            u32 p = i, q = m, o = i;
            while (p < m && q < e) {
                if (sk[q] < sk[p]) {
                    dk[o] = sk[q];
                    dv[o++] = sv[q++];
                } else {
                    dk[o] = sk[p];
                    dv[o++] = sv[p++];
                }
            }
            while (p < m) {
                dk[o] = sk[p];
                dv[o++] = sv[p++];
            }
            while (q < e) {
                dk[o] = sk[q];
                dv[o++] = sv[q++];
            }
        }
        u64* tk = sk;
        sk = dk;
        dk = tk;
        u32* tv = sv;
        sv = dv;
        dv = tv;
    }
    if (sk != k)
        for (u32 i = 0; i < n; ++i) {
            k[i] = sk[i];
            v[i] = sv[i];
        }
}

struct Src {
    u64* buf;
    u64* aux;
    u32 n, cap;
};

// sort and merge duplicate ids (kinds OR-ed); returns the new length
IGN u32 src_dedup(u64* buf, u64* aux, u32 n) {
    if (n == 0) return 0;
    msort64(buf, aux, n);
    u32 o = 0;
    for (u32 i = 0; i < n; ++i) {
        const u64 id = buf[i] >> 8;
        if (o > 0 && (buf[o - 1] >> 8) == id)
            buf[o - 1] |= buf[i] & 0xFF;
        else
            buf[o++] = buf[i];
    }
    return o;
}

IGD void src_add(Shared& sh, Src& s, u32 id, u32 kind) {
    if (s.n == s.cap) {
        s.n = src_dedup(s.buf, s.aux, s.n);
        if (s.n == s.cap) {
            cap_error(sh, IG_CAP_SCRATCH);
            return;
        }
    }
    s.buf[s.n++] = ((u64)id << 8) | kind;
}

// The sources of one instruction: up to 16 in registers (sorted by id, kinds
// OR-ed), spilling to the worker's global list beyond that.
constexpr u32 REG_SRC = 16;
constexpr u32 SS_RECENT = 8;
struct SrcSet {
    u64 r[REG_SRC];
    u32 n;
    bool spilled;
    Src g;
    // the last reader run added (cells of one region often share it)
    u32 run_first, run_n, run_kind;
    // once spilled: the last entries appended, to skip repeats cheaply
    u64 recent[SS_RECENT];
    u32 recent_pos;
};

IGD Src worker_src(DevCtx& c);

IGD void ss_init(DevCtx& c, SrcSet& s) {
    s.n = 0;
    s.spilled = false;
    s.g = worker_src(c);
    s.run_n = 0;
}

// a source set that spills into the given list
IGD void ss_init_buf(SrcSet& s, u64* buf, u64* aux, u32 cap) {
    s.n = 0;
    s.spilled = false;
    s.run_n = 0;
    s.g.buf = buf;
    s.g.aux = aux;
    s.g.n = 0;
    s.g.cap = cap;
}

IGD void ss_add(Shared& sh, SrcSet& s, u32 id, u32 kind) {
    if (s.spilled) {
        // neighbouring cells mostly repeat recent sources
        const u64 key = ((u64)id << 8) | kind;
        bool seen = false;
#pragma unroll
        for (u32 i = 0; i < SS_RECENT; ++i) seen = seen || s.recent[i] == key;
        if (seen) return;
#pragma unroll
        for (u32 i = 0; i < SS_RECENT; ++i)
            if (i == s.recent_pos) s.recent[i] = key;  // static indices keep the ring in registers
        s.recent_pos = (s.recent_pos + 1) % SS_RECENT;
        src_add(sh, s.g, id, kind);
        return;
    }
    bool found = false;
#pragma unroll
    for (u32 i = 0; i < REG_SRC; ++i)
        if (i < s.n && (u32)(s.r[i] >> 8) == id) {
            s.r[i] |= kind;
            found = true;
        }
    if (found) return;
    if (s.n == REG_SRC) {
#pragma unroll
        for (u32 i = 0; i < REG_SRC; ++i) s.g.buf[i] = s.r[i];
        s.g.n = REG_SRC;
        s.spilled = true;
#pragma unroll
        for (u32 i = 0; i < SS_RECENT; ++i) s.recent[i] = ~0ull;
        s.recent_pos = 0;
        src_add(sh, s.g, id, kind);
        return;
    }
    u64 x = ((u64)id << 8) | kind;
    bool shifting = false;  // past the insertion point: shift everything
#pragma unroll
    for (u32 i = 0; i < REG_SRC; ++i) {
        if (i < s.n) {
            if (shifting || s.r[i] > x) {
                shifting = true;
                const u64 t = s.r[i];
                s.r[i] = x;
                x = t;
            }
        } else if (i == s.n) {
            s.r[i] = x;
        }
    }
    s.n += 1;
}

IGD Src worker_src(DevCtx& c) {
    Src s;
    IG_SIM_CHECK(tid() < c.threads, "source scratch per thread");
    s.buf = c.wk_src + (size_t)tid() * c.cap_src;
    s.aux = c.wk_src2 + (size_t)tid() * c.cap_src;
    s.n = 0;
    s.cap = c.cap_src;
    return s;
}

// Stage the edges of instruction x (sources sorted by id, kinds OR-ed).  An
// instruction without any dependency waits for the synchronisation point.
IGN void stage_global(DevCtx& c, Shared& sh, u32 x, u64* buf, u64* aux, u32 n0) {
    const u32 slot = x - sh.unit_first;
    const u32 n = src_dedup(buf, aux, n0);
    const u32 off = atomicAdd(&sh.stage_top, n);
    if ((u64)off + n > (u64)c.cap_unit * 8 || slot >= c.cap_unit) {
        cap_error(sh, IG_CAP_UNIT);
        return;
    }
    for (u32 i = 0; i < n; ++i) {
        const u32 from = (u32)(buf[i] >> 8);
        c.stage_from[off + i] = from;
        c.stage_kind[off + i] = (u8)(buf[i] & 0xFF);
        c.has_succ[from] = 1;
    }
    c.tab_off[slot] = off;
    c.tab_cnt[slot] = n;
}

IGD void stage(DevCtx& c, Shared& sh, u32 x, SrcSet& s) {
    if (s.spilled) {
        stage_global(c, sh, x, s.g.buf, s.g.aux, s.g.n);
        return;
    }
    const u32 slot = x - sh.unit_first;
    if (s.n == 0) {
        s.r[0] = ((u64)sh.s.S << 8) | IG_DEP_SYNC;
        s.n = 1;
    }
    const u32 n = s.n;
    const u32 off = atomicAdd(&sh.stage_top, n);
    if ((u64)off + n > (u64)c.cap_unit * 8 || slot >= c.cap_unit) {
        cap_error(sh, IG_CAP_UNIT);
        return;
    }
#pragma unroll
    for (u32 i = 0; i < REG_SRC; ++i)
        if (i < n) {
            const u32 from = (u32)(s.r[i] >> 8);
            c.stage_from[off + i] = from;
            c.stage_kind[off + i] = (u8)(s.r[i] & 0xFF);
            c.has_succ[from] = 1;
        }
    c.tab_off[slot] = off;
    c.tab_cnt[slot] = n;
}

// Stage the union of a source set and a sorted, duplicate-free list (the
// shared sources of a read group): a two-pointer merge, counted first so the
// staging slot is exact.
IGN void stage_merge_lists(DevCtx& c, Shared& sh, u32 x, const u64* a, u32 na, const u64* b, u32 nb) {
    const u32 slot = x - sh.unit_first;
    u32 n = 0;
    for (u32 i = 0, j = 0; i < na || j < nb; ++n) {
        const u64 ia = i < na ? a[i] >> 8 : ~0ull, jb = j < nb ? b[j] >> 8 : ~0ull;
        if (ia <= jb) ++i;
        if (jb <= ia) ++j;
    }
    const u32 off = atomicAdd(&sh.stage_top, n);
    if ((u64)off + n > (u64)c.cap_unit * 8 || slot >= c.cap_unit) {
        cap_error(sh, IG_CAP_UNIT);
        return;
    }
    u32 o = off;
    for (u32 i = 0, j = 0; i < na || j < nb; ++o) {
        const u64 ia = i < na ? a[i] >> 8 : ~0ull, jb = j < nb ? b[j] >> 8 : ~0ull;
        u32 kind = 0;
        u32 from;
        if (ia <= jb) {
            kind |= (u32)(a[i] & 0xFF);
            from = (u32)ia;
            ++i;
        }
        if (jb <= ia) {
            kind |= (u32)(b[j] & 0xFF);
            from = (u32)jb;
            ++j;
        }
        c.stage_from[o] = from;
        c.stage_kind[o] = (u8)kind;
        c.has_succ[from] = 1;
    }
    c.tab_off[slot] = off;
    c.tab_cnt[slot] = n;
}

IGD void stage_with_list(DevCtx& c, Shared& sh, u32 x, SrcSet& s, const u64* list, u32 nlist) {
    if (nlist == 0) {
        stage(c, sh, x, s);
        return;
    }
    if (s.spilled) {
        const u32 n = src_dedup(s.g.buf, s.g.aux, s.g.n);
        stage_merge_lists(c, sh, x, s.g.buf, n, list, nlist);
        return;
    }
    // the register set goes through the worker's list (sorted already)
    u64* buf = s.g.buf;
#pragma unroll
    for (u32 i = 0; i < REG_SRC; ++i)
        if (i < s.n) buf[i] = s.r[i];
    stage_merge_lists(c, sh, x, buf, s.n, list, nlist);
}

// ===========================================================================
// Instruction records
// ===========================================================================
IGD void put_instr(DevCtx& c, u32 x, u8 kind, u8 flags, u32 task, u32 chunk, u32 buffer, u32 mem, u32 src_mem,
                   u32 alloc, u32 src_alloc, const i64 lo[3], const i64 hi[3]) {
    c.i_kind[x] = kind;
    c.i_flags[x] = flags;
    c.i_mem[x] = (u16)mem;
    c.i_src_mem[x] = (u16)src_mem;
    c.i_task[x] = task;
    c.i_chunk[x] = chunk;
    c.i_buffer[x] = buffer;
    c.i_alloc[x] = alloc;
    c.i_src_alloc[x] = src_alloc;
    const u64 cap = c.cap_instr;
    for (u32 d = 0; d < 3; ++d) {
        c.i_box[d * cap + x] = lo[d];
        c.i_box[(3 + d) * cap + x] = hi[d];
    }
    c.has_succ[x] = 0;
}

// ===========================================================================
// Grids and boxes
// ===========================================================================
IGD const i64* bps(DevCtx& c, const DBuf& B, u32 d) { return WI64(c, B.bp_off[d]); }

IGD u32 bp_find(const i64* a, u32 n, i64 x) {  // exact index or NONE
    u32 lo = 0, hi = n;
    while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < n && a[lo] == x) ? lo : NONE;
}

// Coordinate -> breakpoint index through the grid's hash (1-2 probes).
constexpr i64 HX_EMPTY = (i64)0x8000000000000000ull;
IGD u32 hx_slot(i64 x, u32 bits) { return (u32)(((u64)x * 0x9E3779B97F4A7C15ull) >> (64 - bits)); }

IGD u32 hx_find(DevCtx& c, const DBuf& B, u32 d, i64 x) {
    const u32 bits = B.hx_bits[d], mask = (1u << bits) - 1;
    const u32* t = c.heap + B.hx_off[d];
    for (u32 h = hx_slot(x, bits);; h = (h + 1) & mask) {
        const i64 k = *(const i64*)(t + 4 * h);
        if (k == x) return t[4 * h + 2];
        if (k == HX_EMPTY) return NONE;
    }
}

IGD u32 heap_alloc(DevCtx& c, Shared& sh, u32 words);
IGD void heap_release(DevCtx& c, u32 p);

// (thread 0) rebuild the hash of dimension d after its breakpoints changed
IGN void hx_build(DevCtx& c, Shared& sh, DBuf& B, u32 d) {
    heap_release(c, B.hx_off[d]);
    const u32 n = B.n[d] + 1;
    u32 bits = 2;
    while ((1u << bits) < 2 * n) ++bits;
    B.hx_bits[d] = bits;
    B.hx_off[d] = heap_alloc(c, sh, 4u << bits);
    if (!B.hx_off[d]) return;
    u32* t = c.heap + B.hx_off[d];
    for (u32 h = 0; h < (1u << bits); ++h) *(i64*)(t + 4 * h) = HX_EMPTY;
    const i64* bp = (const i64*)(c.heap + B.bp_off[d]);
    const u32 mask = (1u << bits) - 1;
    for (u32 i = 0; i < n; ++i) {
        u32 h = hx_slot(bp[i], bits);
        while (*(i64*)(t + 4 * h) != HX_EMPTY) h = (h + 1) & mask;
        *(i64*)(t + 4 * h) = bp[i];
        t[4 * h + 2] = i;
    }
}

IGD u32 cell_of(const DBuf& B, u32 i0, u32 i1, u32 i2) { return (i0 * B.n[1] + i1) * B.n[2] + i2; }

IGD u32 alloc_local(const DAlloc& a, u32 i0, u32 i1, u32 i2) {
    return ((i0 - a.clo[0]) * (a.chi[1] - a.clo[1]) + (i1 - a.clo[1])) * (a.chi[2] - a.clo[2]) + (i2 - a.clo[2]);
}

IGD bool box_contains(const i64 olo[3], const i64 ohi[3], const i64 lo[3], const i64 hi[3]) {
    for (u32 d = 0; d < 3; ++d)
        if (lo[d] < olo[d] || hi[d] > ohi[d]) return false;
    return true;
}

IGD bool box_empty(const i64 lo[3], const i64 hi[3]) {
    for (u32 d = 0; d < 3; ++d)
        if (lo[d] >= hi[d]) return true;
    return false;
}

// merge relation of allocation planning: positive-volume overlap or a shared
// face (touching in exactly one dimension, overlapping in the others)
IGD bool box_merges(const i64* a, const i64* b) {
    u32 pos = 0, touch = 0;
    for (u32 d = 0; d < 3; ++d) {
        const i64 hi = a[3 + d] < b[3 + d] ? a[3 + d] : b[3 + d];
        const i64 lo = a[d] > b[d] ? a[d] : b[d];
        const i64 ov = hi - lo;
        if (ov > 0)
            ++pos;
        else if (ov == 0)
            ++touch;
    }
    return pos == 3 || (pos == 2 && touch == 1);
}

IGD bool box6_contains(const i64* o, const i64* b) {
    for (u32 d = 0; d < 3; ++d)
        if (b[d] < o[d] || b[3 + d] > o[3 + d]) return false;
    return true;
}

IGD bool box6_less(const i64* a, const i64* b) {
    for (u32 d = 0; d < 6; ++d)
        if (a[d] != b[d]) return a[d] < b[d];
    return false;
}

// until no two boxes merge: replace merging pairs by their bounding box
// Append a box to a merge list, merging it into the last box when the two
// merge.  The fixpoint of the merge rule is unique (bounding boxes only
// grow, so any two groups that would merge in one order merge in every
// order), which makes merging early a valid step.  Consecutive chunk boxes of
// one device touch along dimension 0, so lists shrink by a factor of the
// chunks per device before the quadratic fixpoint.  false: no room.
IGD bool box_push_merge(i64* bx, u32& n, u32 cap, const i64 lo[3], const i64 hi[3]) {
    const i64 q[6] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
    if (n > 0) {
        i64* a = bx + 6 * (n - 1);
        if (box_merges(a, q)) {
            for (u32 d = 0; d < 3; ++d) {
                a[d] = a[d] < q[d] ? a[d] : q[d];
                a[3 + d] = a[3 + d] > q[3 + d] ? a[3 + d] : q[3 + d];
            }
            return true;
        }
    }
    if (n >= cap) return false;
    for (u32 d = 0; d < 6; ++d) bx[6 * n + d] = q[d];
    ++n;
    return true;
}

IGN u32 merge_fixpoint(i64* bx, u32 n) {
    bool changed = true;
    while (changed) {
        changed = false;
        for (u32 i = 0; i < n; ++i) {
            u32 j = i + 1;
            while (j < n) {
                i64* a = bx + 6 * i;
                i64* b = bx + 6 * j;
                if (box_merges(a, b)) {
                    for (u32 d = 0; d < 3; ++d) {
                        a[d] = a[d] < b[d] ? a[d] : b[d];
                        a[3 + d] = a[3 + d] > b[3 + d] ? a[3 + d] : b[3 + d];
                    }
                    for (u32 d = 0; d < 6; ++d) b[d] = bx[6 * (n - 1) + d];
                    --n;
                    changed = true;
                } else {
                    ++j;
                }
            }
        }
    }
    return n;
}

// Canonical decomposition of a sorted list of linear cell indices: dim-0
// slabs cut where the 2-D cross-section changes, inside a slab dim-1 cut
// where the 1-D cross-section changes, dim-2 maximal runs; boxes in order.
template <class Emit>
IGD u32 canon_cells(const u32* cells, u32 n, u32 n1, u32 n2, Emit emit) {
    const u32 plane = n1 * n2;
    u32 count = 0, p = 0;
    while (p < n) {
        const u32 i0 = cells[p] / plane;
        u32 q = p;
        while (q < n && cells[q] / plane == i0) ++q;
        u32 i0b = i0 + 1, r = q;
        while (r < n) {
            const u32 j0 = cells[r] / plane;
            if (j0 != i0b) break;
            u32 s = r;
            while (s < n && cells[s] / plane == j0) ++s;
            if (s - r != q - p) break;
            bool same = true;
            for (u32 t = 0; t < q - p && same; ++t) same = (cells[p + t] % plane) == (cells[r + t] % plane);
            if (!same) break;
            ++i0b;
            r = s;
        }
        u32 a = p;
        while (a < q) {
            const u32 i1 = (cells[a] % plane) / n2;
            u32 b = a;
            while (b < q && (cells[b] % plane) / n2 == i1) ++b;
            u32 i1b = i1 + 1, cc = b;
            while (cc < q) {
                const u32 j1 = (cells[cc] % plane) / n2;
                if (j1 != i1b) break;
                u32 dd = cc;
                while (dd < q && (cells[dd] % plane) / n2 == j1) ++dd;
                if (dd - cc != b - a) break;
                bool same = true;
                for (u32 t = 0; t < b - a && same; ++t) same = (cells[a + t] % n2) == (cells[cc + t] % n2);
                if (!same) break;
                ++i1b;
                cc = dd;
            }
            u32 e = a;
            while (e < b) {
                const u32 i2 = cells[e] % n2;
                u32 f = e + 1;
                while (f < b && cells[f] % n2 == cells[f - 1] % n2 + 1) ++f;
                emit(i0, i0b, i1, i1b, i2, cells[f - 1] % n2 + 1);
                ++count;
                e = f;
            }
            a = cc;
        }
        p = r;
    }
    return count;
}

// ===========================================================================
// Split (Sec. 3.1) and range mappers (Sec. 2.1, Listing 2)
// ===========================================================================
IGD i64 fpart(i64 n, i64 i, i64 parts) { return (n * i) / parts; }

IGD void chunk_range(const DevCtx& c, i64 lo, i64 hi, u32 k, i64& clo, i64& chi) {
    const u32 K = c.per_dev, dv = k / K, u = k % K, i = dv / c.devices, j = dv % c.devices;
    const i64 n = hi - lo;
    const i64 a = lo + fpart(n, i, c.nodes), b = lo + fpart(n, i + 1, c.nodes);
    const i64 s = a + fpart(b - a, j, c.devices), e = a + fpart(b - a, j + 1, c.devices);
    clo = s + fpart(e - s, u, K);
    chi = s + fpart(e - s, u + 1, K);
}

IGD void map_region(const ig_access& a, const i64 clo[3], const i64 chi[3], const DBuf& B, i64 lo[3], i64 hi[3]) {
    for (u32 d = 0; d < 3; ++d) {
        lo[d] = 0;
        hi[d] = 1;
    }
    for (u32 d = 0; d < B.dims; ++d) {
        switch (a.mapper) {
            case IG_MAP_ONE_TO_ONE:
                lo[d] = clo[d];
                hi[d] = chi[d];
                break;
            case IG_MAP_NEIGHBORHOOD:
                lo[d] = clo[d] - a.radius[d];
                hi[d] = chi[d] + a.radius[d];
                break;
            case IG_MAP_ALL:
                lo[d] = 0;
                hi[d] = B.ext[d];
                break;
            case IG_MAP_SLICE:
                if (d == a.slice_dim) {
                    lo[d] = 0;
                    hi[d] = B.ext[d];
                } else {
                    lo[d] = clo[d];
                    hi[d] = chi[d];
                }
                break;
            default:
                lo[d] = a.fixed.min[d];
                hi[d] = a.fixed.max[d];
                break;
        }
        if (lo[d] < 0) lo[d] = 0;
        if (hi[d] > B.ext[d]) hi[d] = B.ext[d];
    }
}

IGD u32 mem_of_chunk(const DevCtx& c, u32 k) { return 2 + k / c.per_dev; }
IGD u32 owner_of(u32 m) { return m % nt(); }

// live allocation on (b, m) containing a box (0: none)
IGD u32 live_containing(DevCtx& c, u32 b, u32 m, const i64 lo[3], const i64 hi[3]) {
    const u32 base = (b * c.n_mem + m) * MAX_LIVE, n = c.live_n[b * c.n_mem + m];
    for (u32 i = 0; i < n; ++i) {
        const DAlloc& a = c.allocs[c.live[base + i]];
        if (box_contains(a.lo, a.hi, lo, hi)) return c.live[base + i];
    }
    return 0;
}

IGD u32 live_containing_cell(DevCtx& c, u32 b, u32 m, u32 i0, u32 i1, u32 i2) {
    const u32 base = (b * c.n_mem + m) * MAX_LIVE, n = c.live_n[b * c.n_mem + m];
    for (u32 i = 0; i < n; ++i) {
        const DAlloc& a = c.allocs[c.live[base + i]];
        if (i0 >= a.clo[0] && i0 < a.chi[0] && i1 >= a.clo[1] && i1 < a.chi[1] && i2 >= a.clo[2] && i2 < a.chi[2])
            return c.live[base + i];
    }
    return 0;
}

// ===========================================================================
// Regions of the current task: chunk ranges, mapped regions, grid cells.
// Missing grid coordinates are collected for refinement.
// ===========================================================================
IGN void compute_regions(DevCtx& c, Shared& sh) {
    const ig_task_desc& td = c.cmds[sh.t_cmd].task;
    const u32 C = c.chunks, A = sh.t_nacc;
    for (u32 idx = tid(); idx < C * A; idx += nt()) {
        const u32 k = idx / A, j = idx % A;
        Region& r = c.reg[k * IG_MAX_ACCESS + j];
        const ig_access& a = td.access[j];
        r.buffer = a.buffer;
        r.mode = a.mode;
        i64 clo[3] = {0, sh.t_lo[1], sh.t_lo[2]};
        i64 chi[3] = {0, sh.t_hi[1], sh.t_hi[2]};
        chunk_range(c, sh.t_lo[0], sh.t_hi[0], k, clo[0], chi[0]);
        r.empty = box_empty(clo, chi) ? 1u : 0u;
        if (!r.empty) {
            const DBuf& B = c.bufs[a.buffer];
            map_region(a, clo, chi, B, r.lo, r.hi);
            r.empty = box_empty(r.lo, r.hi) ? 1u : 0u;
            if (!r.empty)
                for (u32 d = 0; d < 3; ++d) {
                    const u32 a0 = hx_find(c, B, d, r.lo[d]);
                    const u32 a1 = hx_find(c, B, d, r.hi[d]);
                    r.clo[d] = a0;
                    r.chi[d] = a1;
                    if (a0 == NONE || a1 == NONE) {
                        const u32 slot = atomicAdd(c.miss_n, a0 == NONE && a1 == NONE ? 2u : 1u);
                        u32 s = slot;
                        if (a0 == NONE && s < c.cap_scr) {
                            c.miss_val[s] = r.lo[d];
                            c.miss_bd[s++] = a.buffer * 4 + d;
                        } else if (a0 == NONE) {
                            ++s;
                        }
                        if (a1 == NONE && s < c.cap_scr) {
                            c.miss_val[s] = r.hi[d];
                            c.miss_bd[s] = a.buffer * 4 + d;
                        }
                    }
                }
        }
    }
    bar();
}

// ===========================================================================
// Grid refinement: insert new coordinates into a buffer's grid and move every
// per-cell array of that buffer (buffer map, init, stamps, allocation maps)
// onto the finer grid.  Values are copied, so the represented functions are
// unchanged.
// ===========================================================================
IGN void refine_buffer(DevCtx& c, Shared& sh, u32 b, const u64* keys, u32 lo, u32 hi) {
    DBuf& B = c.bufs[b];
    // --- thread 0: new breakpoints, remap tables, new arrays ---
    if (tid() == 0) {
        u32 newoff[3], newn[3];
        for (u32 d = 0; d < 3; ++d) {
            const i64* old = bps(c, B, d);
            const u32 no = B.n[d] + 1;
            u32 cnt = 0;
            for (u32 i = lo; i < hi; ++i)
                if ((u32)(keys[i] >> 42) == b * 4 + d) ++cnt;
            const u32 nn = no + cnt;
            newoff[d] = heap_alloc(c, sh, 2 * nn);
            if (sh.s.error) break;
            i64* out = WI64(c, newoff[d]);
            u32 p = 0, q = lo, o = 0;
            while (q < hi && (u32)(keys[q] >> 42) != b * 4 + d) ++q;
            while (p < no || (q < hi && (u32)(keys[q] >> 42) == b * 4 + d)) {
                const bool take_new = q < hi && (u32)(keys[q] >> 42) == b * 4 + d &&
                                      (p >= no || (i64)(keys[q] & ((1ull << 42) - 1)) < old[p]);
                if (take_new)
                    out[o++] = (i64)(keys[q++] & ((1ull << 42) - 1));
                else
                    out[o++] = old[p++];
            }
            newn[d] = o - 1;
            if (newn[d] > c.cap_scr) {
                cap_error(sh, IG_CAP_SCRATCH);
                break;
            }
            // old cell of each new cell
            u32 oc = 0;
            for (u32 i = 0; i < newn[d]; ++i) {
                while (oc + 1 < no && old[oc + 1] <= out[i]) ++oc;
                c.remap[d * c.cap_scr + i] = oc;
            }
        }
        if (!sh.s.error) {
            const u32 nc = newn[0] * newn[1] * newn[2];
            sh.scan_tmp[0] = nc;
            // stash old arrays in scan_tmp
            sh.scan_tmp[1] = B.prod_off;
            sh.scan_tmp[2] = B.pm_off;
            sh.scan_tmp[3] = B.mask_off;
            sh.scan_tmp[4] = B.init_off;
            sh.scan_tmp[5] = B.stamp_off;
            sh.scan_tmp[10] = B.wcp_off;
            sh.scan_tmp[11] = B.rcp_off;
            sh.scan_tmp[6] = B.n[0];
            sh.scan_tmp[7] = B.n[1];
            sh.scan_tmp[8] = B.n[2];
            for (u32 d = 0; d < 3; ++d) {
                heap_release(c, B.bp_off[d]);
                B.bp_off[d] = newoff[d];
                B.n[d] = newn[d];
                hx_build(c, sh, B, d);
            }
            B.ncells = nc;
            B.uninit = 0;
            B.prod_off = heap_alloc(c, sh, nc);
            B.pm_off = heap_alloc(c, sh, nc);
            B.mask_off = heap_alloc(c, sh, 2 * nc * c.mw);
            B.init_off = heap_alloc(c, sh, nc);
            B.stamp_off = heap_alloc(c, sh, 2 * nc);
            B.wcp_off = heap_alloc(c, sh, nc);
            B.rcp_off = heap_alloc(c, sh, nc);
            // allocations of this buffer: new cell boxes and arrays
            u32 na = 0;
            for (u32 m = 0; m < c.n_mem; ++m) {
                const u32 base = (b * c.n_mem + m) * MAX_LIVE, n = c.live_n[b * c.n_mem + m];
                for (u32 i = 0; i < n; ++i) {
                    DAlloc& a = c.allocs[c.live[base + i]];
                    c.cons_off[na++] = c.live[base + i];
                    // old geometry goes to the region scratch of this slot
                    Region& sv = c.reg[na - 1];
                    for (u32 d = 0; d < 3; ++d) {
                        sv.clo[d] = a.clo[d];
                        sv.chi[d] = a.chi[d];
                        a.clo[d] = bp_find(bps(c, B, d), B.n[d] + 1, a.lo[d]);
                        a.chi[d] = bp_find(bps(c, B, d), B.n[d] + 1, a.hi[d]);
                    }
                    sv.buffer = a.am_off;
                    a.ncells = (a.chi[0] - a.clo[0]) * (a.chi[1] - a.clo[1]) * (a.chi[2] - a.clo[2]);
                    a.am_off = heap_alloc(c, sh, 4 * a.ncells);
                }
            }
            sh.scan_tmp[9] = na;
        }
    }
    if (failed(sh)) return;
    const u32 nc = sh.scan_tmp[0];
    const u32 on1 = sh.scan_tmp[7], on2 = sh.scan_tmp[8];
    const u32* r0 = c.remap;
    const u32* r1 = c.remap + c.cap_scr;
    const u32* r2 = c.remap + 2 * c.cap_scr;
    // --- buffer-level arrays ---
    for (u32 cell = tid(); cell < nc; cell += nt()) {
        const u32 i2 = cell % B.n[2], i1 = (cell / B.n[2]) % B.n[1], i0 = cell / (B.n[1] * B.n[2]);
        const u32 oc = (r0[i0] * on1 + r1[i1]) * on2 + r2[i2];
        W32(c, B.prod_off)[cell] = W32(c, sh.scan_tmp[1])[oc];
        W32(c, B.pm_off)[cell] = W32(c, sh.scan_tmp[2])[oc];
        for (u32 w = 0; w < c.mw; ++w) W64(c, B.mask_off)[cell * c.mw + w] = W64(c, sh.scan_tmp[3])[oc * c.mw + w];
        const u32 iv = W32(c, sh.scan_tmp[4])[oc];
        W32(c, B.init_off)[cell] = iv;
        if (!iv) atomicAdd(&B.uninit, 1u);
        W64(c, B.stamp_off)[cell] = W64(c, sh.scan_tmp[5])[oc];
        W32(c, B.wcp_off)[cell] = W32(c, sh.scan_tmp[10])[oc];
        W32(c, B.rcp_off)[cell] = W32(c, sh.scan_tmp[11])[oc];
    }
    // --- allocation maps: every thread takes cells of every allocation
    // (each new cell comes from one old cell; reader blocks come from the
    // memory's free list, which any thread may use) ---
    const u32 na = sh.scan_tmp[9];
    for (u32 s = 0; s < na; ++s) {
        const u32 id = c.cons_off[s];
        const DAlloc& a = c.allocs[id];
        const Region& sv = c.reg[s];
        const u32 on1a = sv.chi[1] - sv.clo[1], on2a = sv.chi[2] - sv.clo[2];
        const u32 n1 = a.chi[1] - a.clo[1], n2 = a.chi[2] - a.clo[2];
        AmCell* cells = am_cells(c, a);
        const AmCell* ocl = (const AmCell*)(c.heap + sv.buffer);
        // Refinement only splits cells: the first new cell of an old cell
        // takes over its reader list, the other parts get copies.
        for (u32 l = tid(); l < a.ncells; l += nt()) {
            const u32 i2 = a.clo[2] + l % n2, i1 = a.clo[1] + (l / n2) % n1, i0 = a.clo[0] + l / (n1 * n2);
            const bool f0 = i0 == a.clo[0] || r0[i0 - 1] != r0[i0];
            const bool f1 = i1 == a.clo[1] || r1[i1 - 1] != r1[i1];
            const bool f2 = i2 == a.clo[2] || r2[i2 - 1] != r2[i2];
            const u32 ol = ((r0[i0] - sv.clo[0]) * on1a + (r1[i1] - sv.clo[1])) * on2a + (r2[i2] - sv.clo[2]);
            AmCell e = am_load(ocl + ol);
            if (!(f0 && f1 && f2) && e.ov) e.ov = rd_copy(c, sh, a.mem, e.ov);
            cells[l] = e;
        }
    }
    bar();
    if (tid() == 0) {
        for (u32 s = 1; s <= 5; ++s) heap_release(c, sh.scan_tmp[s]);
        heap_release(c, sh.scan_tmp[10]);
        heap_release(c, sh.scan_tmp[11]);
        for (u32 s = 0; s < na; ++s) heap_release(c, c.reg[s].buffer);
    }
    bar();
}

IGN void refine_all(DevCtx& c, Shared& sh) {
    // thread 0 sorts the missing coordinates (key = buffer*4+dim, value)
    if (tid() == 0) {
        u32 n = *c.miss_n;
        if (n > c.cap_scr) {
            cap_error(sh, IG_CAP_SCRATCH);
            n = 0;
        }
        u64* key = c.wk_key;
        for (u32 i = 0; i < n; ++i) key[i] = ((u64)c.miss_bd[i] << 42) | (u64)c.miss_val[i];
        msort64(key, c.wk_key2, n);
        u32 o = 0;
        for (u32 i = 0; i < n; ++i)
            if (o == 0 || key[o - 1] != key[i]) key[o++] = key[i];
        sh.miss_total = o;
        *c.miss_n = 0;
    }
    bar();
    const u32 n = uniform(sh.miss_total);
    u32 i = 0;
    while (i < n && !failed(sh)) {
        const u32 b = (u32)(c.wk_key[i] >> 44);
        u32 j = i;
        while (j < n && (u32)(c.wk_key[j] >> 44) == b) ++j;
        refine_buffer(c, sh, b, c.wk_key, i, j);
        i = j;
    }
    bar();
}

// ===========================================================================
// Output of a compiled command: staged edges -> edge records in (to, from)
// order.
// ===========================================================================
IGD void unit_begin(DevCtx& c, Shared& sh) {
    if (tid() == 0) {
        sh.unit_first = (u32)sh.s.n_instr;
        sh.unit_n = 0;
        sh.stage_top = 0;
        sh.copy_top = 0;
        sh.nfree = 0;
    }
    bar();
}

IGN void unit_end(DevCtx& c, Shared& sh) {
    rb_stash_return(c, sh);
    if (failed(sh)) return;
    const u32 n = sh.unit_n;
    // per-instruction edge counts -> output offsets
    const u32 total = block_exscan(sh, c.tab_cnt, n);
    if ((u64)sh.s.n_edges + total > c.cap_edges) {
        if (tid() == 0) cap_error(sh, IG_CAP_EDGES);
        bar();
        return;
    }
    const u64 base = sh.s.n_edges;
    for (u32 i = tid(); i < n; i += nt()) {
        const u32 off = c.tab_cnt[i];
        const u32 cnt = (i + 1 < n ? c.tab_cnt[i + 1] : total) - off;
        const u32 src = c.tab_off[i];
        for (u32 e = 0; e < cnt; ++e) {
            c.e_from[base + off + e] = c.stage_from[src + e];
            c.e_kinds[base + off + e] = c.stage_kind[src + e];
            c.e_to[base + off + e] = sh.unit_first + i;
        }
    }
    bar();
    if (tid() == 0) {
        sh.s.n_edges += total;
        sh.s.n_instr += n;
    }
    bar();
}

// ===========================================================================
// Horizons and epochs (Sec. 3.5): SYNC edges from the execution front, i.e.
// every instruction since the last horizon/epoch without a successor.
// ===========================================================================
IGN void compile_sync(DevCtx& c, Shared& sh, bool epoch) {
    tick(c, sh, PH_OTHER);
    if ((u64)sh.s.n_instr + 1 > c.cap_instr) {
        if (tid() == 0) cap_error(sh, IG_CAP_INSTRUCTIONS);
        bar();
        return;
    }
    const u32 x = (u32)sh.s.n_instr;
    const u32 lo = sh.s.last_sync, n = x - lo;
    const u32 T = nt(), t = tid(), per = (n + T - 1) / T;
    const u32 a = lo + (t * per < n ? t * per : n), e = (a + per < x) ? a + per : x;
    u32 cnt = 0;
    for (u32 i = a; i < e; ++i) cnt += c.has_succ[i] ? 0 : 1;
    u32 total;
    const u32 excl = block_excl(sh, cnt, &total);
    if ((u64)sh.s.n_edges + total > c.cap_edges) {
        if (t == 0) cap_error(sh, IG_CAP_EDGES);
        bar();
        return;
    }
    u64 o = sh.s.n_edges + excl;
    for (u32 i = a; i < e; ++i)
        if (!c.has_succ[i]) {
            c.e_from[o] = i;
            c.e_to[o] = x;
            c.e_kinds[o] = IG_DEP_SYNC;
            ++o;
            c.has_succ[i] = 1;
        }
    bar();
    if (t == 0) {
        const i64 z[3] = {0, 0, 0};
        put_instr(c, x, epoch ? IG_EPOCH : IG_HORIZON, 0, NONE, NONE, NONE, 0xFFFF, 0xFFFF, 0, 0, z, z);
        sh.s.n_edges += total;
        sh.s.n_instr += 1;
        if (epoch) {
            sh.s.E = x;
            sh.s.S = x;
            sh.s.pending = NONE;
        } else {
            if (sh.s.pending != NONE) sh.s.S = sh.s.pending;
            sh.s.pending = x;
        }
        sh.s.last_sync = x;
    }
    bar();
    tick(c, sh, PH_SYNC);
}

// ===========================================================================
// Allocation phase (Sec. 3.2).  Per (buffer, memory) whose requirements of
// this task are not all inside a live allocation: merge the live allocations
// with all window requirements on that pair, allocate each resulting box that
// holds an uncovered requirement, copy the up-to-date data of every swallowed
// allocation into it (resize), free the swallowed ones.
// ===========================================================================

// Boxes of the pair (b, m): live allocations and window requirements;
// returns the number of merged boxes in the worker's box scratch, with the
// new ones (holding an uncovered requirement of this task) first, sorted.
IGN u32 plan_pair(DevCtx& c, Shared& sh, u32 b, u32 m, u32& n_new) {
    IG_SIM_CHECK(tid() < c.n_workers, "box scratch per worker");
    i64* bx = c.wk_box + (size_t)tid() * c.cap_box * 6;
    u32 n = 0;
    const u32 lb = (b * c.n_mem + m) * MAX_LIVE, ln = c.live_n[b * c.n_mem + m];
    auto add = [&](const i64* lo, const i64* hi) {
        if (!box_push_merge(bx, n, c.cap_box, lo, hi)) cap_error(sh, IG_CAP_SCRATCH);
    };
    for (u32 i = 0; i < ln; ++i) {
        const DAlloc& a = c.allocs[c.live[lb + i]];
        add(a.lo, a.hi);
    }
    const u32 d = m - 2, A = sh.t_nacc;
    for (u32 k = d * c.per_dev; k < (d + 1) * c.per_dev; ++k)
        for (u32 j = 0; j < A; ++j) {
            const Region& r = c.reg[k * IG_MAX_ACCESS + j];
            if (!r.empty && r.buffer == b) add(r.lo, r.hi);
        }
    // the commands queued behind this task in the current flush
    for (u32 w = 0; w < sh.win_n; ++w) {
        const u32 e = c.queue[sh.win_first + w];
        if (e & 0x80000000u) continue;
        const ig_task_desc& td = c.cmds[e].task;
        for (u32 k = d * c.per_dev; k < (d + 1) * c.per_dev; ++k) {
            i64 clo[3], chi[3];
            chunk_range(c, td.box.min[0], td.box.max[0], k, clo[0], chi[0]);
            clo[1] = td.box.min[1];
            clo[2] = td.box.min[2];
            chi[1] = td.box.max[1];
            chi[2] = td.box.max[2];
            if (box_empty(clo, chi)) continue;
            for (u32 j = 0; j < td.n_access; ++j) {
                if (td.access[j].buffer != b) continue;
                i64 lo[3], hi[3];
                map_region(td.access[j], clo, chi, c.bufs[b], lo, hi);
                if (!box_empty(lo, hi)) add(lo, hi);
            }
        }
    }
    n = merge_fixpoint(bx, n);
    // new boxes: those containing an uncovered requirement of this task
    u32 nn = 0;
    for (u32 i = 0; i < n; ++i) {
        bool hit = false;
        for (u32 k = d * c.per_dev; k < (d + 1) * c.per_dev && !hit; ++k)
            for (u32 j = 0; j < A && !hit; ++j) {
                const Region& r = c.reg[k * IG_MAX_ACCESS + j];
                if (r.empty || r.buffer != b) continue;
                i64 rb6[6] = {r.lo[0], r.lo[1], r.lo[2], r.hi[0], r.hi[1], r.hi[2]};
                if (!box6_contains(bx + 6 * i, rb6)) continue;
                if (live_containing(c, b, m, r.lo, r.hi) == 0) hit = true;
            }
        if (hit) {
            for (u32 t = 0; t < 6; ++t) {
                const i64 v = bx[6 * nn + t];
                bx[6 * nn + t] = bx[6 * i + t];
                bx[6 * i + t] = v;
            }
            ++nn;
        }
    }
    // insertion sort of the new boxes by their minimum (lexicographic)
    for (u32 i = 1; i < nn; ++i)
        for (u32 j = i; j > 0 && box6_less(bx + 6 * j, bx + 6 * (j - 1)); --j)
            for (u32 t = 0; t < 6; ++t) {
                const i64 v = bx[6 * j + t];
                bx[6 * j + t] = bx[6 * (j - 1) + t];
                bx[6 * (j - 1) + t] = v;
            }
    n_new = nn;
    return n;
}

// cells of allocation `a` that are up to date on memory m, sorted
IGN u32 utd_cells(DevCtx& c, Shared& sh, const DAlloc& a, u32 m, u32* out) {
    const DBuf& B = c.bufs[a.buffer];
    const u64* mask = W64(c, B.mask_off);
    u32 n = 0;
    for (u32 i0 = a.clo[0]; i0 < a.chi[0]; ++i0)
        for (u32 i1 = a.clo[1]; i1 < a.chi[1]; ++i1)
            for (u32 i2 = a.clo[2]; i2 < a.chi[2]; ++i2) {
                const u32 cell = cell_of(B, i0, i1, i2);
                if ((mask[cell * c.mw + (m >> 6)] >> (m & 63)) & 1) {
                    if (n >= c.cap_scr) {
                        cap_error(sh, IG_CAP_SCRATCH);
                        return n;
                    }
                    out[n++] = cell;
                }
            }
    return n;
}

// sorted ids of the live allocations of (b, m) inside box q
IGD u32 absorbed_of(DevCtx& c, u32 b, u32 m, const i64* q, u32* out) {
    const u32 lb = (b * c.n_mem + m) * MAX_LIVE, ln = c.live_n[b * c.n_mem + m];
    u32 n = 0;
    for (u32 i = 0; i < ln; ++i) {
        const DAlloc& a = c.allocs[c.live[lb + i]];
        const i64 ab[6] = {a.lo[0], a.lo[1], a.lo[2], a.hi[0], a.hi[1], a.hi[2]};
        if (box6_contains(q, ab)) out[n++] = c.live[lb + i];
    }
    for (u32 i = 1; i < n; ++i)
        for (u32 j = i; j > 0 && out[j] < out[j - 1]; --j) {
            const u32 v = out[j];
            out[j] = out[j - 1];
            out[j - 1] = v;
        }
    return n;
}

// ---------------------------------------------------------------------------
// Allocation-map cells: edges against the state before an instruction and the
// updates after it (owner-only).
// ---------------------------------------------------------------------------
// a read: dataflow edge from the last writer, lifetime if that is the ALLOC
IGD void cell_read_edge(Shared& sh, SrcSet& s, const AmCell& e) {
    const u32 w = e.w & ~W_ALLOC;
    if (w < sh.s.S)
        ss_add(sh, s, sh.s.S, IG_DEP_TRUE);
    else
        ss_add(sh, s, w, (e.w & W_ALLOC) ? IG_DEP_LIFETIME : IG_DEP_TRUE);
}

IGD void writer_edge(Shared& sh, SrcSet& s, const AmCell& e, u32 kind) {
    const u32 w = e.w & ~W_ALLOC;
    if (w < sh.s.S)
        ss_add(sh, s, sh.s.S, kind);
    else
        ss_add(sh, s, w, (e.w & W_ALLOC) ? IG_DEP_LIFETIME : kind);
}

// edges of kind from the readers first..first+n-1 (as eff_r maps each);
// true if any reader still exists
IGD bool reader_run_edges(Shared& sh, SrcSet& s, u32 first, u32 n, u32 kind) {
    const u32 end = first + n, S = sh.s.S, E = sh.s.E;
    u32 lo = first < E ? E : first;
    if (lo >= end) return false;
    if (n > 1) {
        if (s.run_n == n && s.run_first == first && s.run_kind == kind) return true;  // added already
        s.run_first = first;
        s.run_n = n;
        s.run_kind = kind;
    }
    if (lo < S) {
        ss_add(sh, s, S, kind);
        lo = S;
    }
    for (u32 r = lo; r < end; ++r) ss_add(sh, s, r, kind);
    return true;
}

// a write: anti edges from the readers, else an output edge from the writer
IGD void cell_write_edge(DevCtx& c, Shared& sh, SrcSet& s, const AmCell& e) {
    bool any = false;
    u32 x;
    if (e.r0 != NONE && eff_r(sh, e.r0, x)) {
        ss_add(sh, s, x, IG_DEP_ANTI);
        any = true;
    }
    if (e.r1 != NONE && eff_r(sh, e.r1, x)) {
        ss_add(sh, s, x, IG_DEP_ANTI);
        any = true;
    }
    rd_each(c, e.ov, [&](u32 first, u32 n) { any |= reader_run_edges(sh, s, first, n, IG_DEP_ANTI); });
    if (!any) writer_edge(sh, s, e, IG_DEP_OUTPUT);
}

IGD void cell_free_edges(DevCtx& c, Shared& sh, SrcSet& s, const AmCell& e) {
    const u32 w = e.w & ~W_ALLOC;
    ss_add(sh, s, w < sh.s.S ? sh.s.S : w, IG_DEP_LIFETIME);
    u32 x;
    if (e.r0 != NONE && eff_r(sh, e.r0, x)) ss_add(sh, s, x, IG_DEP_LIFETIME);
    if (e.r1 != NONE && eff_r(sh, e.r1, x)) ss_add(sh, s, x, IG_DEP_LIFETIME);
    rd_each(c, e.ov, [&](u32 first, u32 n) { reader_run_edges(sh, s, first, n, IG_DEP_LIFETIME); });
}

// readers gain x (inline slots first; slots whose reader reads as absent or
// duplicates the other slot's synchronisation point are reused); e is the
// record at p as loaded
IGD void cell_add_reader_at(DevCtx& c, Shared& sh, u32 m, AmCell* p, AmCell e, u32 x) {
    if (e.r0 != NONE && e.r0 < sh.s.E) e.r0 = NONE;
    if (e.r1 != NONE && e.r1 < sh.s.E) e.r1 = NONE;
    if (e.r0 != NONE && e.r1 != NONE && e.r0 < sh.s.S && e.r1 < sh.s.S) e.r1 = NONE;
    if (e.r0 == NONE) {
        p->r0 = x;
        p->r1 = e.r1;
    } else if (e.r1 == NONE) {
        p->r0 = e.r0;
        p->r1 = x;
    } else {
        rd_append(c, sh, m, &p->ov, x);
    }
}

IGD void cell_add_reader(DevCtx& c, Shared& sh, u32 m, AmCell* p, u32 x) {
    cell_add_reader_at(c, sh, m, p, am_load(p), x);
}

// a write: new last writer, no readers (e: the record at p as loaded)
IGD void cell_set_writer_at(DevCtx& c, u32 m, AmCell* p, const AmCell& e, u32 w) {
    AmCell n;
    n.w = w;
    n.r0 = NONE;
    n.r1 = NONE;
    n.ov = 0;
#ifdef IG_HOST_SIM
    *p = n;
#else
    *(uint4*)p = make_uint4(n.w, n.r0, n.r1, n.ov);
#endif
    if (e.ov) {
        u32 h = e.ov;
        rd_clear(c, m, &h);
    }
}

IGD void cell_set_writer(DevCtx& c, u32 m, AmCell* p, u32 w) { cell_set_writer_at(c, m, p, am_load(p), w); }

// Visit the cells [clo, chi) (grid indices) of allocation a, loading their
// records eight at a time so that the loads are in flight together: f(e, p)
// gets the record as it was before the visit and its address.
constexpr u32 CELL_BATCH = 8;
template <class F>
IGD void scan_cells(AmCell* cl, const DAlloc& a, const u32 clo[3], const u32 chi[3], F f) {
    const u32 n1 = chi[1] - clo[1], n2 = chi[2] - clo[2];
    const u32 total = (chi[0] - clo[0]) * n1 * n2;
    for (u32 base = 0; base < total; base += CELL_BATCH) {
        AmCell e[CELL_BATCH];
        AmCell* ptr[CELL_BATCH];
#pragma unroll
        for (u32 q = 0; q < CELL_BATCH; ++q) {
            const u32 t = base + q < total ? base + q : total - 1;
            const u32 i2 = t % n2, i1 = (t / n2) % n1, i0 = t / (n1 * n2);
            ptr[q] = cl + alloc_local(a, clo[0] + i0, clo[1] + i1, clo[2] + i2);
            e[q] = am_load(ptr[q]);
        }
#pragma unroll
        for (u32 q = 0; q < CELL_BATCH; ++q)
            if (base + q < total) f(e[q], ptr[q]);
    }
}

// The same visit restricted to the grid columns i0 = g (mod G) of the box:
// the G members of a team each take one residue, so every cell is visited
// by exactly one member.
template <class F>
IGD void scan_cells_cols(AmCell* cl, const DAlloc& a, const u32 clo[3], const u32 chi[3], u32 g, u32 G, F f) {
    const u32 i0f = clo[0] + (g + G - clo[0] % G) % G;
    if (i0f >= chi[0]) return;
    const u32 n0 = (chi[0] - 1 - i0f) / G + 1, n1 = chi[1] - clo[1], n2 = chi[2] - clo[2];
    const u32 total = n0 * n1 * n2;
    for (u32 base = 0; base < total; base += CELL_BATCH) {
        AmCell e[CELL_BATCH];
        AmCell* ptr[CELL_BATCH];
#pragma unroll
        for (u32 q = 0; q < CELL_BATCH; ++q) {
            const u32 t = base + q < total ? base + q : total - 1;
            const u32 i2 = t % n2, i1 = (t / n2) % n1, j0 = t / (n1 * n2);
            ptr[q] = cl + alloc_local(a, i0f + j0 * G, clo[1] + i1, clo[2] + i2);
            e[q] = am_load(ptr[q]);
        }
#pragma unroll
        for (u32 q = 0; q < CELL_BATCH; ++q)
            if (base + q < total) f(e[q], ptr[q]);
    }
}

IGD void cell_init(AmCell* p, u32 w) {
    p->w = w;
    p->r0 = NONE;
    p->r1 = NONE;
    p->ov = 0;
}

IGD void free_edges(DevCtx& c, Shared& sh, SrcSet& s, const DAlloc& a) {
    scan_cells(am_cells(c, a), a, a.clo, a.chi, [&](const AmCell& e, AmCell*) { cell_free_edges(c, sh, s, e); });
}

IGN void release_readers(DevCtx& c, const DAlloc& a) {
    scan_cells(am_cells(c, a), a, a.clo, a.chi, [&](const AmCell& e, AmCell* p) {
        if (e.ov) rd_clear(c, a.mem, &p->ov);
    });
}

IGD void live_remove(DevCtx& c, u32 b, u32 m, u32 id) {
    const u32 lb = (b * c.n_mem + m) * MAX_LIVE;
    u32& ln = c.live_n[b * c.n_mem + m];
    for (u32 i = 0; i < ln; ++i)
        if (c.live[lb + i] == id) {
            c.live[lb + i] = c.live[lb + ln - 1];
            --ln;
            return;
        }
}

IGN void free_stage_one(DevCtx& c, Shared& sh, u32 x, const DAlloc& a, u64* bm);

IGN void alloc_phase(DevCtx& c, Shared& sh) {
    const u32 NP = sh.s.n_buffers * c.n_mem, A = sh.t_nacc, C = c.chunks;
    for (u32 i = tid(); i < NP; i += nt()) {
        c.pair_flag[i] = 0;
        c.pair_cnt[i] = 0;
        c.pair_acnt[i] = 0;
    }
    if (tid() == 0) sh.flag = 0;
    bar();
    for (u32 idx = tid(); idx < C * A; idx += nt()) {
        const u32 k = idx / A, j = idx % A;
        const Region& r = c.reg[k * IG_MAX_ACCESS + j];
        if (r.empty) continue;
        const u32 m = mem_of_chunk(c, k);
        if (live_containing(c, r.buffer, m, r.lo, r.hi) == 0) {
            c.pair_flag[r.buffer * c.n_mem + m] = 1;
            sh.flag = 1;
        }
    }
    if (!uniform(sh.flag)) {
        if (tid() == 0) sh.n_alloc_instr = 0;
        bar();
        return;
    }
    // counting pass, per memory worker
    u32* absorb = c.wk_val + (size_t)tid() * c.cap_scr;
    u32* cells = c.wk_val2 + (size_t)tid() * c.cap_scr;
    const i64* bx = c.wk_box + (size_t)tid() * c.cap_box * 6;
    for (u32 m = tid(); m < c.n_mem; m += nt()) {
        if (m < 2) continue;
        for (u32 b = 0; b < sh.s.n_buffers; ++b) {
            if (!c.pair_flag[b * c.n_mem + m]) continue;
            u32 nn;
            plan_pair(c, sh, b, m, nn);
            u32 cnt = 0;
            for (u32 i = 0; i < nn; ++i) {
                const u32 na = absorbed_of(c, b, m, bx + 6 * i, absorb);
                cnt += 1 + na;
                for (u32 q = 0; q < na; ++q) {
                    const u32 nc = utd_cells(c, sh, c.allocs[absorb[q]], m, cells);
                    cnt += canon_cells(cells, nc, c.bufs[b].n[1], c.bufs[b].n[2],
                                       [](u32, u32, u32, u32, u32, u32) {});
                }
            }
            c.pair_cnt[b * c.n_mem + m] = cnt;
            c.pair_acnt[b * c.n_mem + m] = nn;
        }
    }
    bar();
    const u32 total = block_exscan(sh, c.pair_cnt, NP);
    const u32 total_allocs = block_exscan(sh, c.pair_acnt, NP);
    if (tid() == 0) {
        if (sh.unit_first + total > c.cap_instr) cap_error(sh, IG_CAP_INSTRUCTIONS);
        if (sh.s.next_alloc + total_allocs > c.cap_allocs) cap_error(sh, IG_CAP_ALLOCS);
        if (total > c.cap_unit) cap_error(sh, IG_CAP_UNIT);
    }
    if (failed(sh)) return;
    // the new allocations' geometry -> thread 0 creates their map arrays
    for (u32 m = tid(); m < c.n_mem; m += nt()) {
        if (m < 2) continue;
        for (u32 b = 0; b < sh.s.n_buffers; ++b) {
            if (!c.pair_flag[b * c.n_mem + m]) continue;
            u32 nn;
            plan_pair(c, sh, b, m, nn);
            for (u32 i = 0; i < nn; ++i) {
                DAlloc& na = c.allocs[sh.s.next_alloc + c.pair_acnt[b * c.n_mem + m] + i];
                const DBuf& B = c.bufs[b];
                na.buffer = b;
                na.mem = m;
                na.alive = 1;
                for (u32 d = 0; d < 3; ++d) {
                    na.lo[d] = bx[6 * i + d];
                    na.hi[d] = bx[6 * i + 3 + d];
                    na.clo[d] = bp_find(bps(c, B, d), B.n[d] + 1, na.lo[d]);
                    na.chi[d] = bp_find(bps(c, B, d), B.n[d] + 1, na.hi[d]);
                }
                na.ncells = (na.chi[0] - na.clo[0]) * (na.chi[1] - na.clo[1]) * (na.chi[2] - na.clo[2]);
            }
        }
    }
    bar();
    if (tid() == 0) {
        for (u32 i = 0; i < total_allocs; ++i) {
            DAlloc& na = c.allocs[sh.s.next_alloc + i];
            na.am_off = heap_alloc(c, sh, 4 * na.ncells);
        }
    }
    if (failed(sh)) return;
    // emission pass
    for (u32 m = tid(); m < c.n_mem; m += nt()) {
        if (m < 2) continue;
        for (u32 b = 0; b < sh.s.n_buffers; ++b) {
            if (!c.pair_flag[b * c.n_mem + m]) continue;
            u32 nn;
            plan_pair(c, sh, b, m, nn);
            u32 x = sh.unit_first + c.pair_cnt[b * c.n_mem + m];
            const DBuf& B = c.bufs[b];
            for (u32 i = 0; i < nn; ++i) {
                const u32 nid = sh.s.next_alloc + c.pair_acnt[b * c.n_mem + m] + i;
                DAlloc& na = c.allocs[nid];
                const u32 xa = x++;
                put_instr(c, xa, IG_ALLOC, 0, sh.t_id, NONE, b, m, 0xFFFF, nid, 0, na.lo, na.hi);
                SrcSet s0;
                ss_init(c, s0);
                stage(c, sh, xa, s0);
                AmCell* ncl = am_cells(c, na);
                for (u32 l = 0; l < na.ncells; ++l) cell_init(ncl + l, xa | W_ALLOC);
                const u32 nabs = absorbed_of(c, b, m, bx + 6 * i, absorb);
                for (u32 q = 0; q < nabs; ++q) {
                    const DAlloc& old = c.allocs[absorb[q]];
                    AmCell* ocl = am_cells(c, old);
                    const u32 nc = utd_cells(c, sh, old, m, cells);
                    canon_cells(cells, nc, B.n[1], B.n[2], [&](u32 a0, u32 a1, u32 b0, u32 b1, u32 c0, u32 c1) {
                        const u32 xc = x++;
                        i64 lo[3] = {bps(c, B, 0)[a0], bps(c, B, 1)[b0], bps(c, B, 2)[c0]};
                        i64 hi[3] = {bps(c, B, 0)[a1], bps(c, B, 1)[b1], bps(c, B, 2)[c1]};
                        put_instr(c, xc, IG_COPY, IG_F_RESIZE, sh.t_id, NONE, b, m, m, nid, absorb[q], lo, hi);
                        SrcSet s;
                        ss_init(c, s);
                        const u32 blo[3] = {a0, b0, c0}, bhi[3] = {a1, b1, c1};
                        scan_cells(ocl, old, blo, bhi, [&](const AmCell& e, AmCell*) { cell_read_edge(sh, s, e); });
                        scan_cells(ncl, na, blo, bhi, [&](const AmCell& e, AmCell*) { cell_write_edge(c, sh, s, e); });
                        stage(c, sh, xc, s);
                        scan_cells(ocl, old, blo, bhi,
                                   [&](const AmCell& e, AmCell* p) { cell_add_reader_at(c, sh, m, p, e, xc); });
                        scan_cells(ncl, na, blo, bhi,
                                   [&](const AmCell& e, AmCell* p) { cell_set_writer_at(c, m, p, e, xc); });
                    });
                }
                for (u32 q = 0; q < nabs; ++q) {
                    DAlloc& old = c.allocs[absorb[q]];
                    const u32 xf = x++;
                    put_instr(c, xf, IG_FREE, 0, sh.t_id, NONE, b, m, 0xFFFF, absorb[q], 0, old.lo, old.hi);
                    free_stage_one(c, sh, xf, old, c.wk_key + (size_t)tid() * c.cap_scr);
                    release_readers(c, old);
                    old.alive = 0;
                    live_remove(c, b, m, absorb[q]);
                    const u32 slot = atomicAdd(&sh.nfree, 1u);
                    c.miss_bd[slot] = absorb[q];  // freed: arrays released below
                }
                const u32 lb = (b * c.n_mem + m) * MAX_LIVE;
                u32& ln = c.live_n[b * c.n_mem + m];
                if (ln >= MAX_LIVE) {
                    cap_error(sh, IG_CAP_LIVE);
                } else {
                    c.live[lb + ln] = nid;
                    ++ln;
                }
            }
        }
    }
    bar();
    if (tid() == 0) {
        for (u32 i = 0; i < sh.nfree; ++i) {
            DAlloc& old = c.allocs[c.miss_bd[i]];
            heap_release(c, old.am_off);
            old.am_off = 0;
        }
        sh.s.resizes += sh.nfree;
        sh.s.next_alloc += total_allocs;
        sh.n_alloc_instr = total;
        sh.unit_n += total;
        sh.nfree = 0;
    }
    bar();
}

// ===========================================================================
// Coherence (Sec. 3.3).  Counting pass: per memory worker, consumers in
// (chunk, access) order; stale cells grouped by (producer memory, original
// producer, source allocation); canonical boxes; the memory is marked up to
// date at once (consumer split).
// ===========================================================================
// Emit the copies of one consumer from its stale cells, grouped: cells[g..h)
// share one key (producer memory, original producer, source allocation).
IGD u32 emit_groups(DevCtx& c, Shared& sh, const u64* key, const u32* val, u32 n, const DBuf& B, u32 k, u32 j,
                    u32 b, u32 dst, u32 m, u32 off, bool write) {
    u32 o = off, cnt = 0;
    for (u32 g = 0; g < n;) {
        u32 h = g;
        while (h < n && key[h] == key[g]) ++h;
        const u32 pm = (u32)(key[g] >> 56);
        const u32 src = (u32)(key[g] & 0xFFFFFF);
        const u32 nb = canon_cells(val + g, h - g, B.n[1], B.n[2], [&](u32 a0, u32 a1, u32 b0, u32 b1, u32 c0, u32 c1) {
            if (!write) return;
            CopyRec& cr = c.copies[o++];
            cr.chunk = k;
            cr.pad0 = k * IG_MAX_ACCESS + j;
            cr.buffer = b;
            cr.src_alloc = src;
            cr.dst_alloc = dst;
            cr.src_mem = pm;
            cr.dst_mem = m;
            cr.clo[0] = a0;
            cr.chi[0] = a1;
            cr.clo[1] = b0;
            cr.chi[1] = b1;
            cr.clo[2] = c0;
            cr.chi[2] = c1;
        });
        if (write) atomicAdd(&c.inbox_cnt[pm], nb);
        cnt += nb;
        g = h;
    }
    return cnt;
}

// ===========================================================================
// Coherence (Sec. 3.3).  Counting pass: per memory worker, consumers in
// (chunk, access) order; stale cells grouped by (producer memory, original
// producer, source allocation); canonical boxes; the memory is marked up to
// date at once (consumer split).  Up to 16 stale cells of a consumer are
// kept sorted in registers; more go through the worker's global scratch.
// ===========================================================================
constexpr u32 REG_NEED = 16;

// Thread teams: with several threads per simulated device, the G threads of a
// team (consecutive, within one wave) share one memory's large scans.  G is
// the largest power of two (at most 64) with G * n_dev <= threads; memories
// are taken in passes of threads / G.
IGD u32 team_size(const DevCtx& c) {
    u32 g = 1;
    while (g < 64 && 2 * g * c.n_dev <= nt()) g <<= 1;
    return g;
}

// Without direct device-to-device copies (staging), a copy between two
// devices of one node becomes two instructions, through pinned host memory.
IGD bool copy_staged(const DevCtx& c, u32 src_mem, u32 dst_mem) {
    return c.staging && src_mem >= 2 && (src_mem - 2) / c.devices == (dst_mem - 2) / c.devices;
}

// Copies of the records [off, off + n) that are staged.
IGD u32 staged_among(const DevCtx& c, u32 off, u32 n) {
    u32 st = 0;
    if (c.staging)
        for (u32 q = off; q < off + n; ++q) st += copy_staged(c, c.copies[q].src_mem, c.copies[q].dst_mem);
    return st;
}

IGN void coherence_count(DevCtx& c, Shared& sh) {
    const u32 A = sh.t_nacc, K = c.per_dev;
    const u32 G = team_size(c);
    // A read with no cell that is stale on its memory and holds data at the
    // start of the task needs no copy whatever the consumers before it copy
    // (copies only add memories to the masks): such reads are found by all
    // threads at once and skipped by the ordered pass below (cons_x: 0).
    for (u32 q = tid(); q < c.chunks * A; q += nt()) {
        const u32 k = q / A, j = q % A, idx = k * IG_MAX_ACCESS + j;
        const Region& r = c.reg[idx];
        u32 stale = 0;
        if (!r.empty && (r.mode & IG_READ)) {
            const u32 m = mem_of_chunk(c, k);
            const DBuf& B = c.bufs[r.buffer];
            const u64* mask = W64(c, B.mask_off);
            for (u32 i0 = r.clo[0]; i0 < r.chi[0] && !stale; ++i0)
                for (u32 i1 = r.clo[1]; i1 < r.chi[1] && !stale; ++i1)
                    for (u32 i2 = r.clo[2]; i2 < r.chi[2]; ++i2) {
                        const u64* mk = mask + (size_t)cell_of(B, i0, i1, i2) * c.mw;
                        if ((mk[m >> 6] >> (m & 63)) & 1) continue;
                        u64 any = 0;
                        for (u32 w = 0; w < c.mw; ++w) any |= mk[w];
                        if (any) {
                            stale = 1;
                            break;
                        }
                    }
        }
        c.cons_x[idx] = stale;
    }
    bar();
    for (u32 m = tid(); m < c.n_mem; m += nt()) {
        if (m < 2) continue;
        const u32 d = m - 2;
        u32 nbig = 0;  // large reads of this memory deferred to coherence_big
        IG_SIM_CHECK(tid() < c.n_workers, "coherence scratch per worker");
        u64* key = c.wk_key + (size_t)tid() * c.cap_scr;
        u32* val = c.wk_val + (size_t)tid() * c.cap_scr;
        u64* key2 = c.wk_key2 + (size_t)tid() * c.cap_scr;
        u32* val2 = c.wk_val2 + (size_t)tid() * c.cap_scr;
        u64* lkey = sh.wkey + (size_t)tid() * REG_NEED;
        u32* lval = sh.wval + (size_t)tid() * REG_NEED;
        u32 total = 0, kcount = 0;
        // The last two read regions scanned on this memory: after a scan
        // every cell of the region is up to date on m (or holds no data), so
        // the same region again needs no copies.
        u32 seen[2][7];
        u32 n_seen = 0;
        for (u32 k = d * K; k < (d + 1) * K; ++k) {
            i64 k0, k1;
            chunk_range(c, sh.t_lo[0], sh.t_hi[0], k, k0, k1);
            const bool chunk_empty = k0 >= k1 || sh.t_lo[1] >= sh.t_hi[1] || sh.t_lo[2] >= sh.t_hi[2];
            if (!chunk_empty) ++kcount;
            for (u32 j = 0; j < A; ++j) {
                const u32 idx = k * IG_MAX_ACCESS + j;
                c.cons_cnt[idx] = 0;
                c.cons_off[idx] = 0;
                const Region& r = c.reg[idx];
                if (chunk_empty || r.empty || !(r.mode & IG_READ) || !c.cons_x[idx]) continue;
                const u32 b = r.buffer;
                const u32 key7[7] = {b, r.clo[0], r.clo[1], r.clo[2], r.chi[0], r.chi[1], r.chi[2]};
                bool again = false;
#pragma unroll
                for (u32 q = 0; q < 2; ++q) {
                    bool eq = q < n_seen;
#pragma unroll
                    for (u32 t = 0; t < 7; ++t) eq = eq && seen[q][t] == key7[t];
                    again = again || eq;
                }
                if (again) continue;
#pragma unroll
                for (u32 t = 0; t < 7; ++t) {
                    seen[1][t] = seen[0][t];
                    seen[0][t] = key7[t];
                }
                n_seen = n_seen < 2 ? n_seen + 1 : 2;
                // A large read deferred to the team scan makes its cells up
                // to date there, after this loop; a later read of the same
                // buffer must find them covered already (the consumer split
                // in (chunk, access) order), so it skips them here, or is
                // skipped whole when the deferred region contains it.
                u32 nex = 0;
                u32 exlo[MAX_BIG][3], exhi[MAX_BIG][3];
                bool inside = false;
#pragma unroll
                for (u32 q = 0; q < MAX_BIG; ++q) {
                    if (q >= nbig) break;
                    const Region& D = c.reg[c.big_idx[m * MAX_BIG + q]];
                    if (D.buffer != b) continue;
                    bool cont = true, meet = true;
#pragma unroll
                    for (u32 t3 = 0; t3 < 3; ++t3) {
                        cont = cont && D.clo[t3] <= r.clo[t3] && r.chi[t3] <= D.chi[t3];
                        meet = meet && D.clo[t3] < r.chi[t3] && r.clo[t3] < D.chi[t3];
                    }
                    inside = inside || cont;
                    if (!cont && meet) {
#pragma unroll
                        for (u32 e = 0; e < MAX_BIG; ++e)
                            if (e == nex)
#pragma unroll
                                for (u32 t3 = 0; t3 < 3; ++t3) {
                                    exlo[e][t3] = D.clo[t3];
                                    exhi[e][t3] = D.chi[t3];
                                }
                        ++nex;
                    }
                }
                if (inside) continue;
                const u32 ncr = (r.chi[0] - r.clo[0]) * (r.chi[1] - r.clo[1]) * (r.chi[2] - r.clo[2]);
                if (G > 1 && ncr >= BIG_CELLS && nbig < MAX_BIG) {
                    c.big_idx[m * MAX_BIG + nbig] = idx;
                    ++nbig;
                    continue;
                }
                const DBuf& B = c.bufs[b];
                const u32* prod = W32(c, B.prod_off);
                const u32* pmv = W32(c, B.pm_off);
                u64* mask = W64(c, B.mask_off);
                u64 rk[REG_NEED];
                u32 rv[REG_NEED];
                u32 n = 0;
                bool big = false;
                bool ordered = true;  // keys seen in non-decreasing order (then no sort is needed)
                u64 last_key = 0;
                // the last source allocation found, reused while cells stay inside it
                u32 l_pm = NONE, l_src = 0, l_lo[3] = {0, 0, 0}, l_hi[3] = {0, 0, 0};
                for (u32 i0 = r.clo[0]; i0 < r.chi[0]; ++i0)
                    for (u32 i1 = r.clo[1]; i1 < r.chi[1]; ++i1)
                        for (u32 i2 = r.clo[2]; i2 < r.chi[2]; ++i2) {
                            if (nex) {
                                bool ex = false;
#pragma unroll
                                for (u32 e = 0; e < MAX_BIG; ++e)
                                    ex = ex || (e < nex && i0 >= exlo[e][0] && i0 < exhi[e][0] && i1 >= exlo[e][1] &&
                                                i1 < exhi[e][1] && i2 >= exlo[e][2] && i2 < exhi[e][2]);
                                if (ex) continue;
                            }
                            const u32 cell = cell_of(B, i0, i1, i2);
                            const u64* mk = mask + (size_t)cell * c.mw;
                            if ((mk[m >> 6] >> (m & 63)) & 1) continue;
                            u64 any = 0;
                            for (u32 w = 0; w < c.mw; ++w) any |= mk[w];
                            if (!any) continue;  // never initialised: nothing to copy
                            const u32 pm = pmv[cell];
                            const u32 p = eff_w(sh, prod[cell]);
                            u32 src;
                            if (pm == l_pm && i0 >= l_lo[0] && i0 < l_hi[0] && i1 >= l_lo[1] && i1 < l_hi[1] &&
                                i2 >= l_lo[2] && i2 < l_hi[2]) {
                                src = l_src;
                            } else {
                                src = live_containing_cell(c, b, pm, i0, i1, i2);
                                if (src == 0) {
                                    set_error(sh, IG_E_INTERNAL);
                                } else {
                                    const DAlloc& sa = c.allocs[src];
                                    l_pm = pm;
                                    l_src = src;
                                    for (u32 t3 = 0; t3 < 3; ++t3) {
                                        l_lo[t3] = sa.clo[t3];
                                        l_hi[t3] = sa.chi[t3];
                                    }
                                }
                            }
                            u64 x = ((u64)pm << 56) | ((u64)p << 24) | (u64)(src & 0xFFFFFF);
                            if (x < last_key) ordered = false;
                            last_key = x;
                            if (!big && n == REG_NEED) {
#pragma unroll
                                for (u32 i = 0; i < REG_NEED; ++i) {
                                    key[i] = rk[i];
                                    val[i] = rv[i];
                                }
                                big = true;
                            }
                            if (big) {
                                if (n >= c.cap_scr) {
                                    cap_error(sh, IG_CAP_SCRATCH);
                                    continue;
                                }
                                key[n] = x;
                                val[n] = cell;
                            } else {
                                // sorted insertion, stable: equal keys keep cell order
                                u32 y = cell;
                                bool shifting = false;  // past the insertion point: shift everything
#pragma unroll
                                for (u32 i = 0; i < REG_NEED; ++i) {
                                    if (i < n) {
                                        if (shifting || rk[i] > x) {
                                            shifting = true;
                                            const u64 tk = rk[i];
                                            rk[i] = x;
                                            x = tk;
                                            const u32 tv = rv[i];
                                            rv[i] = y;
                                            y = tv;
                                        }
                                    } else if (i == n) {
                                        rk[i] = x;
                                        rv[i] = y;
                                    }
                                }
                            }
                            ++n;
                        }
                if (n == 0) continue;
                const u32 dst = live_containing(c, b, m, r.lo, r.hi);
                if (dst == 0) set_error(sh, IG_E_INTERNAL);
                const u64* gk;
                const u32* gv;
                if (big) {
                    if (!ordered) msort_kv(key, val, key2, val2, n);
                    gk = key;
                    gv = val;
                } else {
#pragma unroll
                    for (u32 i = 0; i < REG_NEED; ++i)
                        if (i < n) {
                            lkey[i] = rk[i];
                            lval[i] = rv[i];
                        }
                    gk = lkey;
                    gv = lval;
                }
                const u32 cnt = emit_groups(c, sh, gk, gv, n, B, k, j, b, dst, m, 0, false);
                const u32 off = atomicAdd(&sh.copy_top, cnt);
                if (off + cnt > c.cap_unit) {
                    cap_error(sh, IG_CAP_UNIT);
                    continue;
                }
                emit_groups(c, sh, gk, gv, n, B, k, j, b, dst, m, off, true);
                // consumer split: the data is now present on m
                for (u32 i = 0; i < n; ++i) atomicOr(&mask[(size_t)gv[i] * c.mw + (m >> 6)], 1ull << (m & 63));
                c.cons_off[idx] = off;
                c.cons_cnt[idx] = cnt;
                total += cnt + staged_among(c, off, cnt);  // instructions
            }
        }
        c.dev_cnt[d] = total;
        c.kdev_cnt[d] = kcount;
        c.big_n[m] = nbig;
    }
}

// The key of a stale cell (producer memory, original producer, source
// allocation), as in coherence_count; 0 with an error when no live
// allocation on the producer memory holds the cell.
struct SrcCache {
    u32 pm, src, lo[3], hi[3];
};

IGD u64 stale_key(DevCtx& c, Shared& sh, SrcCache& l, u32 b, u32 pm, u32 p, u32 i0, u32 i1, u32 i2) {
    if (!(pm == l.pm && i0 >= l.lo[0] && i0 < l.hi[0] && i1 >= l.lo[1] && i1 < l.hi[1] && i2 >= l.lo[2] &&
          i2 < l.hi[2])) {
        const u32 src = live_containing_cell(c, b, pm, i0, i1, i2);
        if (src == 0) {
            set_error(sh, IG_E_INTERNAL);
            return 0;
        }
        const DAlloc& sa = c.allocs[src];
        l.pm = pm;
        l.src = src;
        for (u32 t3 = 0; t3 < 3; ++t3) {
            l.lo[t3] = sa.clo[t3];
            l.hi[t3] = sa.chi[t3];
        }
    }
    return ((u64)pm << 56) | ((u64)p << 24) | (u64)(l.src & 0xFFFFFF);
}

// Large reads deferred by coherence_count, scanned by the team of their
// memory: round r takes every memory's r-th deferred read (in (chunk, access)
// order), so each sees the up-to-date state its predecessors left.
//  1. each member scans a contiguous part of the region's cells (cell order)
//     and keeps its stale cells' (key, cell) pairs;
//  2. the parts are concatenated in member order (block scan), which is the
//     cell order of one sequential scan, and sorted stably by key if needed;
//  3. members take contiguous parts of the list, emit the groups that start
//     in their part (canonical boxes, block scan of the counts for the copy
//     slots) and mark the copied cells up to date.
IGN void coherence_big(DevCtx& c, Shared& sh) {
    if (tid() == 0) sh.flag = 0;
    bar();
    for (u32 m = tid() + 2; m < c.n_mem; m += nt()) atomicMax(&sh.flag, c.big_n[m]);
    const u32 rounds = uniform(sh.flag);
    if (rounds == 0) return;
    const u32 G = team_size(c), TP = nt() / G, ts = tid() / G, g = tid() % G;
    const u32 seg = c.cap_scr / G;
    for (u32 rnd = 0; rnd < rounds; ++rnd) {
        for (u32 base = 0; base < c.n_dev; base += TP) {
            const u32 d = base + ts, m = d + 2;
            const bool act = d < c.n_dev && rnd < c.big_n[m];
            const u32 w = m % nt();  // the memory's worker: its scratch arrays
            IG_SIM_CHECK(!act || w < c.n_workers, "team scratch per worker");
            u64* key = c.wk_key + (size_t)w * c.cap_scr;
            u32* val = c.wk_val + (size_t)w * c.cap_scr;
            u64* key2 = c.wk_key2 + (size_t)w * c.cap_scr;
            u32* val2 = c.wk_val2 + (size_t)w * c.cap_scr;
            u32* tm = c.tm + 4 * (size_t)m;
            u32 idx = 0, k = 0, j = 0, b = 0, n_g = 0;
            bool ordered = true;
            Region r;
            if (act) {
                idx = c.big_idx[m * MAX_BIG + rnd];
                k = idx / IG_MAX_ACCESS;
                j = idx % IG_MAX_ACCESS;
                r = c.reg[idx];
                b = r.buffer;
                if (g == 0) tm[2] = 0;
                const u32 n1 = r.chi[1] - r.clo[1], n2 = r.chi[2] - r.clo[2];
                const u32 total = (r.chi[0] - r.clo[0]) * n1 * n2;
                if (total > G * seg) cap_error(sh, IG_CAP_SCRATCH);
                const u32 per = (total + G - 1) / G;
                const u32 q0 = g * per < total ? g * per : total;
                const u32 q1 = q0 + per < total ? q0 + per : total;
                const DBuf& B = c.bufs[b];
                const u32* prod = W32(c, B.prod_off);
                const u32* pmv = W32(c, B.pm_off);
                const u64* mask = W64(c, B.mask_off);
                u64* mk_out = key + (size_t)g * seg;
                u32* mv_out = val + (size_t)g * seg;
                SrcCache l;
                l.pm = NONE;
                u64 last = 0;
                u32 i2 = q0 % n2, i1 = (q0 / n2) % n1, i0 = q0 / (n1 * n2);
                for (u32 q = q0; q < q1 && !sh.s.error; ++q) {
                    const u32 a0 = r.clo[0] + i0, a1 = r.clo[1] + i1, a2 = r.clo[2] + i2;
                    if (++i2 == n2) {
                        i2 = 0;
                        if (++i1 == n1) {
                            i1 = 0;
                            ++i0;
                        }
                    }
                    const u32 cell = cell_of(B, a0, a1, a2);
                    const u64* mk = mask + (size_t)cell * c.mw;
                    if ((mk[m >> 6] >> (m & 63)) & 1) continue;
                    u64 any = 0;
                    for (u32 x = 0; x < c.mw; ++x) any |= mk[x];
                    if (!any) continue;
                    const u64 x = stale_key(c, sh, l, b, pmv[cell], eff_w(sh, prod[cell]), a0, a1, a2);
                    if (x < last) ordered = false;
                    last = x;
                    mk_out[n_g] = x;
                    mv_out[n_g] = cell;
                    ++n_g;
                }
            }
            u32 tot;
            const u32 excl = block_excl(sh, act ? n_g : 0, &tot);
            if (act && g == 0) tm[0] = excl;
            bar();
            const u32 off = act ? excl - tm[0] : 0;
            if (act) {
                if (g == G - 1) tm[1] = off + n_g;
                if (!ordered) atomicOr(&tm[2], 1u);
                for (u32 i = 0; i < n_g; ++i) {
                    key2[off + i] = key[(size_t)g * seg + i];
                    val2[off + i] = val[(size_t)g * seg + i];
                }
            }
            bar();
            const u32 n = act ? tm[1] : 0;
            if (act && g > 0 && n_g > 0 && off > 0 && key2[off - 1] > key2[off]) atomicOr(&tm[2], 1u);
            bar();
            if (act && g == 0 && tm[2] && n > 1 && !sh.s.error) msort_kv(key2, val2, key, val, n);
            if (failed(sh)) return;
            // groups starting in this member's part of the list
            u32 gs = 0, ge = 0, cnt = 0, dst = 0;
            if (act && n > 0) {
                const u32 per = (n + G - 1) / G;
                const u32 e0 = g * per < n ? g * per : n, e1 = e0 + per < n ? e0 + per : n;
                gs = e0;
                while (gs < e1 && gs > 0 && key2[gs] == key2[gs - 1]) ++gs;
                ge = gs;
                if (gs < e1) {
                    ge = e1;
                    while (ge < n && key2[ge] == key2[ge - 1]) ++ge;
                }
                dst = live_containing(c, b, m, r.lo, r.hi);
                if (dst == 0) set_error(sh, IG_E_INTERNAL);
                cnt = emit_groups(c, sh, key2 + gs, val2 + gs, ge - gs, c.bufs[b], k, j, b, dst, m, 0, false);
            }
            const u32 excl2 = block_excl(sh, act ? cnt : 0, &tot);
            if (act && g == 0) tm[0] = excl2;
            bar();
            const u32 boff = act ? excl2 - tm[0] : 0;
            if (act && g == G - 1) tm[1] = boff + cnt;
            bar();
            if (act && g == 0) {
                const u32 all = tm[1];
                const u32 at = atomicAdd(&sh.copy_top, all);
                if (at + all > c.cap_unit) cap_error(sh, IG_CAP_UNIT);
                tm[3] = at;
                c.cons_off[idx] = at;
                c.cons_cnt[idx] = all;
                c.dev_cnt[d] += all;
            }
            if (failed(sh)) return;
            if (act && ge > gs) {
                const DBuf& B = c.bufs[b];
                emit_groups(c, sh, key2 + gs, val2 + gs, ge - gs, B, k, j, b, dst, m, tm[3] + boff, true);
                const u32 st = staged_among(c, tm[3] + boff, cnt);  // the second halves of staged copies
                if (st) atomicAdd(&c.dev_cnt[d], st);
                u64* mask = W64(c, B.mask_off);
                for (u32 e = gs; e < ge; ++e) atomicOr(&mask[(size_t)val2[e] * c.mw + (m >> 6)], 1ull << (m & 63));
            }
            bar();
        }
    }
}

// A staged copy: device -> M1 (reads the source), then M1 -> device (writes
// the destination, after the first), ids x and x + 1.  Kept out of line so
// that the direct copies' code keeps its registers.
IGN void emit_staged_copy(DevCtx& c, Shared& sh, const CopyRec& cr, u32 x, const i64 lo[3], const i64 hi[3]) {
    const u32 m = cr.dst_mem;
    const DAlloc& sa = c.allocs[cr.src_alloc];
    const DAlloc& da = c.allocs[cr.dst_alloc];
    AmCell* dcl = am_cells(c, da);
    put_instr(c, x, IG_COPY, 0, sh.t_id, cr.chunk, cr.buffer, 1, cr.src_mem, 0, cr.src_alloc, lo, hi);
    SrcSet s;
    ss_init(c, s);
    scan_cells(am_cells(c, sa), sa, cr.clo, cr.chi, [&](const AmCell& e, AmCell*) { cell_read_edge(sh, s, e); });
    stage(c, sh, x, s);
    put_instr(c, x + 1, IG_COPY, 0, sh.t_id, cr.chunk, cr.buffer, m, 1, cr.dst_alloc, 0, lo, hi);
    SrcSet s2;
    ss_init(c, s2);
    ss_add(sh, s2, x, IG_DEP_TRUE);
    scan_cells(dcl, da, cr.clo, cr.chi, [&](const AmCell& e, AmCell*) { cell_write_edge(c, sh, s2, e); });
    stage(c, sh, x + 1, s2);
    scan_cells(dcl, da, cr.clo, cr.chi, [&](const AmCell& e, AmCell* p) { cell_set_writer_at(c, m, p, e, x + 1); });
}

// Emission pass: ids, records, edges, updates of the destination maps; the
// reads of source allocations go to their owners' inboxes.
IGN void coherence_emit(DevCtx& c, Shared& sh, u32 copy_first) {
    const u32 A = sh.t_nacc, K = c.per_dev;
    // instruction order: per device, (chunk, access), then canonical box
    for (u32 m = tid(); m < c.n_mem; m += nt()) {
        if (m < 2) continue;
        const u32 d = m - 2;
        // instruction offsets within the device: a staged copy takes two
        u32 run = 0;
        for (u32 k = d * K; k < (d + 1) * K; ++k)
            for (u32 j = 0; j < A; ++j) {
                const u32 idx = k * IG_MAX_ACCESS + j;
                c.cons_x[idx] = run;
                if (!c.staging) {
                    run += c.cons_cnt[idx];
                    continue;
                }
                const u32 q0 = c.cons_off[idx], q1 = q0 + c.cons_cnt[idx];
                for (u32 q = q0; q < q1; ++q) {
                    c.copies[q].pad1 = run;
                    run += copy_staged(c, c.copies[q].src_mem, m) ? 2 : 1;
                }
            }
    }
    bar();
    // Copies are independent: their destination cells are disjoint (each
    // stale cell is copied once), their source cells are up to date where
    // they are read and so are no copy's destination, and readers of the
    // sources go to the owners' inboxes.  Any thread takes any copy.
    // Each thread takes a contiguous block of copies: neighbouring copies
    // mostly go to the same memory, and the lanes of a wave would otherwise
    // all return reader blocks to that memory's free list at once.
    const u32 n = sh.copy_top, per = (n + nt() - 1) / nt();
    const u32 q0 = tid() * per, q1 = q0 + per < n ? q0 + per : n;
    for (u32 q = q0; q < q1; ++q) {
        const CopyRec& cr = c.copies[q];
        const u32 m = cr.dst_mem, idx = cr.pad0;
        const u32 x = copy_first + c.dev_base[m - 2] + (c.staging ? cr.pad1 : c.cons_x[idx] + (q - c.cons_off[idx]));
        const DBuf& B = c.bufs[cr.buffer];
        const DAlloc& sa = c.allocs[cr.src_alloc];
        const DAlloc& da = c.allocs[cr.dst_alloc];
        const i64 lo[3] = {bps(c, B, 0)[cr.clo[0]], bps(c, B, 1)[cr.clo[1]], bps(c, B, 2)[cr.clo[2]]};
        const i64 hi[3] = {bps(c, B, 0)[cr.chi[0]], bps(c, B, 1)[cr.chi[1]], bps(c, B, 2)[cr.chi[2]]};
        const bool inter = cr.src_mem >= 2 && (cr.src_mem - 2) / c.devices != (m - 2) / c.devices;
        AmCell* dcl = am_cells(c, da);
        if (copy_staged(c, cr.src_mem, m)) {
            emit_staged_copy(c, sh, cr, x, lo, hi);
        } else {
            put_instr(c, x, IG_COPY, inter ? IG_F_INTER_NODE : 0, sh.t_id, cr.chunk, cr.buffer, m, cr.src_mem,
                      cr.dst_alloc, cr.src_alloc, lo, hi);
            SrcSet s;
            ss_init(c, s);
            scan_cells(am_cells(c, sa), sa, cr.clo, cr.chi,
                       [&](const AmCell& e, AmCell*) { cell_read_edge(sh, s, e); });
            scan_cells(dcl, da, cr.clo, cr.chi, [&](const AmCell& e, AmCell*) { cell_write_edge(c, sh, s, e); });
            stage(c, sh, x, s);
            scan_cells(dcl, da, cr.clo, cr.chi,
                       [&](const AmCell& e, AmCell* p) { cell_set_writer_at(c, m, p, e, x); });
        }
        const u32 slot = atomicAdd(&c.inbox_cur[cr.src_mem], 1u);
        InboxRec& ib = c.inbox[slot];
        ib.alloc = cr.src_alloc;
        ib.reader = x;
        for (u32 t = 0; t < 3; ++t) {
            ib.clo[t] = cr.clo[t];
            ib.chi[t] = cr.chi[t];
        }
    }
}

// The copies' readers of source allocations, memory by memory: the threads
// t with t % n_mem == m form memory m's team, member g taking the grid
// columns i0 = g (mod G) of every record's region, records in inbox order
// (a cell's readers are only ever added by its one owner).
IGN void inbox_drain(DevCtx& c, Shared& sh) {
    const u32 nm = c.n_mem, t = tid();
    const bool teams = nt() >= nm;
    const u32 m0 = teams ? t % nm : t, mstep = teams ? nm : nt();
    const u32 g = teams ? t / nm : 0, G = teams ? (nt() - m0 + nm - 1) / nm : 1;
    for (u32 m = m0; m < nm; m += mstep) {
        const u32 lo = c.inbox_off[m], hi = lo + c.inbox_cnt[m];
        for (u32 q = lo; q < hi; ++q) {
            const InboxRec& ib = c.inbox[q];
            const DAlloc& a = c.allocs[ib.alloc];
            const u32 x = ib.reader;
            scan_cells_cols(am_cells(c, a), a, ib.clo, ib.chi, g, G,
                            [&](const AmCell& e, AmCell* p) { cell_add_reader_at(c, sh, m, p, e, x); });
        }
        if (teams) break;
    }
}

// ===========================================================================
// Device kernels, bindings, buffer-map update (Sec. 3.1, 3.2)
// ===========================================================================
// Pure reads of a buffer the task does not write see the same writers in
// every kernel of the task (kernels change only the cells they write), so
// consecutive kernels of one device reading the same region share one scan
// of its cells, and their reader entries go in as one run of ids, added
// after the device's last kernel (nothing in between looks at them).
IGD bool same_cells(const RdGroup& g, u32 alloc, const Region& rg) {
    return g.alloc == alloc && g.clo[0] == rg.clo[0] && g.clo[1] == rg.clo[1] && g.clo[2] == rg.clo[2] &&
           g.chi[0] == rg.chi[0] && g.chi[1] == rg.chi[1] && g.chi[2] == rg.chi[2];
}

IGD void rd_group_flush(DevCtx& c, Shared& sh, u32 m, RdGroup& g) {
    const DAlloc& a = c.allocs[g.alloc];
    const u32 first = g.first, n = g.n;
    scan_cells(am_cells(c, a), a, g.clo, g.chi, [&](const AmCell& e, AmCell* p) {
        if (n == 1)
            cell_add_reader_at(c, sh, m, p, e, first);
        else
            rd_append_range(c, sh, m, &p->ov, first, n);
    });
    g.n = 0;
}

IGN void kernels_emit_seq(DevCtx& c, Shared& sh, u32 kern_first) {
    const u32 A = sh.t_nacc, K = c.per_dev;
    for (u32 m = tid(); m < c.n_mem; m += nt()) {
        if (m < 2) continue;
        const u32 d = m - 2;
        IG_SIM_CHECK(tid() < c.n_workers, "read-group scratch per worker");
        RdGroup* grp = c.wk_grp + (size_t)tid() * RD_CACHE;
        for (u32 q = 0; q < RD_CACHE; ++q) grp[q].n = 0;
        u32 r = 0;
        for (u32 k = d * K; k < (d + 1) * K; ++k) {
            i64 lo[3] = {0, sh.t_lo[1], sh.t_lo[2]};
            i64 hi[3] = {0, sh.t_hi[1], sh.t_hi[2]};
            chunk_range(c, sh.t_lo[0], sh.t_hi[0], k, lo[0], hi[0]);
            if (box_empty(lo, hi)) continue;
            const u32 x = kern_first + c.kdev_base[d] + r;
            const u64 bi = sh.s.n_binds + (u64)(c.kdev_base[d] + r) * A;
            ++r;
            put_instr(c, x, IG_KERNEL, 0, sh.t_id, k, NONE, m, 0xFFFF, 0, 0, lo, hi);
            u32 al[IG_MAX_ACCESS];
            for (u32 j = 0; j < A; ++j) {
                const Region& rg = c.reg[k * IG_MAX_ACCESS + j];
                al[j] = rg.empty ? 0 : live_containing(c, rg.buffer, m, rg.lo, rg.hi);
                if (!rg.empty && al[j] == 0) set_error(sh, IG_E_INTERNAL);
                c.b_instr[bi + j] = x;
                c.b_access[bi + j] = j;
                c.b_alloc[bi + j] = al[j];
            }
            SrcSet s;
            ss_init(c, s);
            u32 grouped = 0;  // accesses handled by a read group
            const u64* glist = nullptr;  // one group's shared sources, merged at staging
            u32 nglist = 0;
            for (u32 j = 0; j < A; ++j) {
                if (!al[j]) continue;
                const Region& rg = c.reg[k * IG_MAX_ACCESS + j];
                const DAlloc& a = c.allocs[al[j]];
                const u32 mode = rg.mode;
                if (j < RD_CACHE && mode == IG_READ && !((sh.t_wbufs >> rg.buffer) & 1)) {
                    grouped |= 1u << j;
                    RdGroup& g = grp[j];
                    u64* src = c.wk_rsrc + ((size_t)tid() * RD_CACHE + j) * c.cap_src;
                    if (g.n && g.first + g.n == x && same_cells(g, al[j], rg)) {
                        if (!glist) {
                            glist = src;
                            nglist = g.nsrc;
                        } else {
                            for (u32 i = 0; i < g.nsrc; ++i) ss_add(sh, s, (u32)(src[i] >> 8), (u32)(src[i] & 0xFF));
                        }
                        ++g.n;
                        continue;
                    }
                    if (g.n) rd_group_flush(c, sh, m, g);
                    // the sources of this read alone, kept for the next kernels
                    SrcSet t;
                    ss_init_buf(t, src, c.wk_src2 + (size_t)tid() * c.cap_src, c.cap_src);
                    scan_cells(am_cells(c, a), a, rg.clo, rg.chi,
                               [&](const AmCell& e, AmCell*) { cell_read_edge(sh, t, e); });
                    u32 ns;
                    if (!t.spilled) {
#pragma unroll
                        for (u32 i = 0; i < REG_SRC; ++i)
                            if (i < t.n) src[i] = t.r[i];
                        ns = t.n;
                    } else {
                        ns = src_dedup(src, t.g.aux, t.g.n);
                    }
                    if (!glist) {
                        glist = src;
                        nglist = ns;
                    } else {
                        for (u32 i = 0; i < ns; ++i) ss_add(sh, s, (u32)(src[i] >> 8), (u32)(src[i] & 0xFF));
                    }
                    g.alloc = al[j];
                    g.first = x;
                    g.n = 1;
                    g.nsrc = ns;
                    for (u32 t3 = 0; t3 < 3; ++t3) {
                        g.clo[t3] = rg.clo[t3];
                        g.chi[t3] = rg.chi[t3];
                    }
                    continue;
                }
                scan_cells(am_cells(c, a), a, rg.clo, rg.chi, [&](const AmCell& e, AmCell*) {
                    if (mode & IG_READ) cell_read_edge(sh, s, e);
                    if (mode & IG_WRITE) cell_write_edge(c, sh, s, e);
                });
            }
            stage_with_list(c, sh, x, s, glist, nglist);
            // reads first, then writes (a cell both read and written ends written)
            for (u32 j = 0; j < A; ++j) {
                const Region& rg = c.reg[k * IG_MAX_ACCESS + j];
                if (!al[j] || !(rg.mode & IG_READ) || ((grouped >> j) & 1)) continue;
                const DAlloc& a = c.allocs[al[j]];
                scan_cells(am_cells(c, a), a, rg.clo, rg.chi,
                           [&](const AmCell& e, AmCell* p) { cell_add_reader_at(c, sh, m, p, e, x); });
            }
            for (u32 j = 0; j < A; ++j) {
                const Region& rg = c.reg[k * IG_MAX_ACCESS + j];
                if (!al[j] || !(rg.mode & IG_WRITE)) continue;
                const DAlloc& a = c.allocs[al[j]];
                const DBuf& B = c.bufs[rg.buffer];
                u32* prod = W32(c, B.prod_off);
                u32* pmv = W32(c, B.pm_off);
                u64* mask = W64(c, B.mask_off);
                scan_cells(am_cells(c, a), a, rg.clo, rg.chi,
                           [&](const AmCell& e, AmCell* p) { cell_set_writer_at(c, m, p, e, x); });
                for (u32 i0 = rg.clo[0]; i0 < rg.chi[0]; ++i0)
                    for (u32 i1 = rg.clo[1]; i1 < rg.chi[1]; ++i1)
                        for (u32 i2 = rg.clo[2]; i2 < rg.chi[2]; ++i2) {
                            const u32 cell = cell_of(B, i0, i1, i2);
                            prod[cell] = x;
                            pmv[cell] = m;
                            for (u32 w = 0; w < c.mw; ++w)
                                mask[(size_t)cell * c.mw + w] = (w == (m >> 6)) ? (1ull << (m & 63)) : 0ull;
                        }
            }
        }
        for (u32 q = 0; q < RD_CACHE; ++q)
            if (grp[q].n) rd_group_flush(c, sh, m, grp[q]);
    }
}

// The same records when every access to a buffer the task writes stays in its
// chunk's dim-0 range.  Then no cell is touched by two kernels of the task
// unless both only read it, so every kernel sees the task's starting state on
// the cells it accesses (reads see writers, which only the cell's own chunk
// changes; writes see readers, which no other chunk adds to written cells),
// and its edges and writes do not depend on the others.
//  1. any thread takes any kernel: record, bindings, edges, writes;
//  2. reader additions, split by cell among the threads of each device, in
//     kernel order per cell (a cell the kernel itself wrote gets no reader).
// The shared source list of grouped access j on device d (t_gmask): in the
// worker scratch of the device's memory; its length in c.tm.
IGD u64* group_list(DevCtx& c, u32 m, u32 j) {
    return c.wk_rsrc + ((size_t)(m % nt()) * RD_CACHE + j) * c.cap_src;
}

IGN void kernels_emit_par(DevCtx& c, Shared& sh, u32 kern_first) {
    const u32 A = sh.t_nacc, K = c.per_dev, C = c.chunks;
    const u32 gmask = sh.t_gmask;
    // kernel rank of each chunk within its device (empty chunks have none)
    for (u32 d = tid(); d < c.n_dev; d += nt()) {
        u32 r = 0;
        for (u32 k = d * K; k < (d + 1) * K; ++k) {
            i64 k0, k1;
            chunk_range(c, sh.t_lo[0], sh.t_hi[0], k, k0, k1);
            const bool empty = k0 >= k1 || sh.t_lo[1] >= sh.t_hi[1] || sh.t_lo[2] >= sh.t_hi[2];
            c.k_rank[k] = empty ? NONE : r++;
        }
    }
    // grouped reads: one scan of the shared region per (device, access),
    // sources sorted and de-duplicated once for all kernels of the device
    if (gmask) {
        for (u32 w = tid(); w < c.n_dev * RD_CACHE; w += nt()) {
            const u32 d = w / RD_CACHE, j = w % RD_CACHE, m = d + 2;
            if (!((gmask >> j) & 1)) continue;
            IG_SIM_CHECK(m % nt() < c.n_workers, "group lists per worker");
            c.tm[4 * m + j] = 0;
            if (c.kdev_cnt[d] == 0) continue;  // no kernel on the device
            const Region& rg = c.reg[(d * K) * IG_MAX_ACCESS + j];
            u32 kk = d * K;  // the first chunk of the device with a region
            while (kk < (d + 1) * K && c.reg[kk * IG_MAX_ACCESS + j].empty) ++kk;
            if (kk == (d + 1) * K) continue;
            const Region& rk = kk == d * K ? rg : c.reg[kk * IG_MAX_ACCESS + j];
            const u32 al = live_containing(c, rk.buffer, m, rk.lo, rk.hi);
            if (!al) {
                set_error(sh, IG_E_INTERNAL);
                continue;
            }
            const DAlloc& a = c.allocs[al];
            u64* src = group_list(c, m, j);
            SrcSet t;
            ss_init_buf(t, src, c.wk_src2 + (size_t)tid() * c.cap_src, c.cap_src);
            scan_cells(am_cells(c, a), a, rk.clo, rk.chi, [&](const AmCell& e, AmCell*) { cell_read_edge(sh, t, e); });
            u32 ns;
            if (!t.spilled) {
#pragma unroll
                for (u32 i = 0; i < REG_SRC; ++i)
                    if (i < t.n) src[i] = t.r[i];
                ns = t.n;
            } else {
                ns = src_dedup(src, t.g.aux, t.g.n);
            }
            c.tm[4 * m + j] = ns;
        }
    }
    bar();
    // kernel i of the walk is chunk k of device i mod n_dev: the lanes of a
    // wave work on different devices (and free lists)
    for (u32 i = tid(); i < C; i += nt()) {
        const u32 k = (i % c.n_dev) * K + i / c.n_dev;
        const u32 rk = c.k_rank[k];
        if (rk == NONE) continue;
        const u32 d = k / K, m = d + 2;
        i64 lo[3] = {0, sh.t_lo[1], sh.t_lo[2]};
        i64 hi[3] = {0, sh.t_hi[1], sh.t_hi[2]};
        chunk_range(c, sh.t_lo[0], sh.t_hi[0], k, lo[0], hi[0]);
        const u32 x = kern_first + c.kdev_base[d] + rk;
        const u64 bi = sh.s.n_binds + (u64)(c.kdev_base[d] + rk) * A;
        put_instr(c, x, IG_KERNEL, 0, sh.t_id, k, NONE, m, 0xFFFF, 0, 0, lo, hi);
        // per-thread allocation ids in LDS (the coherence keys are free in
        // this phase): a private array indexed by access would live in scratch
        u32* al = reinterpret_cast<u32*>(sh.wkey) + tid() * IG_MAX_ACCESS;
        for (u32 j = 0; j < A; ++j) {
            const Region& rg = c.reg[k * IG_MAX_ACCESS + j];
            al[j] = rg.empty ? 0 : live_containing(c, rg.buffer, m, rg.lo, rg.hi);
            if (!rg.empty && al[j] == 0) set_error(sh, IG_E_INTERNAL);
            c.b_instr[bi + j] = x;
            c.b_access[bi + j] = j;
            c.b_alloc[bi + j] = al[j];
        }
        SrcSet s;
        ss_init(c, s);
        const u64* glist = nullptr;  // the first grouped access's list, merged at staging
        u32 nglist = 0;
        for (u32 j = 0; j < A; ++j) {
            if (!al[j]) continue;
            if ((gmask >> j) & 1) {
                const u64* gl = group_list(c, m, j);
                const u32 ng = c.tm[4 * m + j];
                if (!glist) {
                    glist = gl;
                    nglist = ng;
                } else {
                    for (u32 i = 0; i < ng; ++i) ss_add(sh, s, (u32)(gl[i] >> 8), (u32)(gl[i] & 0xFF));
                }
                continue;
            }
            const Region& rg = c.reg[k * IG_MAX_ACCESS + j];
            const DAlloc& a = c.allocs[al[j]];
            const u32 mode = rg.mode;
            scan_cells(am_cells(c, a), a, rg.clo, rg.chi, [&](const AmCell& e, AmCell*) {
                if (mode & IG_READ) cell_read_edge(sh, s, e);
                if (mode & IG_WRITE) cell_write_edge(c, sh, s, e);
            });
        }
        stage_with_list(c, sh, x, s, glist, nglist);
        for (u32 j = 0; j < A; ++j) {
            const Region& rg = c.reg[k * IG_MAX_ACCESS + j];
            if (!al[j] || !(rg.mode & IG_WRITE)) continue;
            const DAlloc& a = c.allocs[al[j]];
            const DBuf& B = c.bufs[rg.buffer];
            u32* prod = W32(c, B.prod_off);
            u32* pmv = W32(c, B.pm_off);
            u64* mask = W64(c, B.mask_off);
            scan_cells(am_cells(c, a), a, rg.clo, rg.chi,
                       [&](const AmCell& e, AmCell* p) { cell_set_writer_at(c, m, p, e, x); });
            for (u32 i0 = rg.clo[0]; i0 < rg.chi[0]; ++i0)
                for (u32 i1 = rg.clo[1]; i1 < rg.chi[1]; ++i1)
                    for (u32 i2 = rg.clo[2]; i2 < rg.chi[2]; ++i2) {
                        const u32 cell = cell_of(B, i0, i1, i2);
                        prod[cell] = x;
                        pmv[cell] = m;
                        for (u32 w = 0; w < c.mw; ++w)
                            mask[(size_t)cell * c.mw + w] = (w == (m >> 6)) ? (1ull << (m & 63)) : 0ull;
                    }
        }
    }
    bar();
    // reader additions: the threads t with t % n_dev == d share device d's
    // cells, member g taking the grid columns i0 = g (mod G) of every
    // region, each in kernel order
    const u32 nd = c.n_dev, t = tid();
    const u32 d0 = nt() >= nd ? t % nd : t;
    const u32 dstep = nt() >= nd ? nd : nt();
    const u32 g = nt() >= nd ? t / nd : 0;
    const u32 G = nt() >= nd ? (nt() - d0 + nd - 1) / nd : 1;
    auto own_cells = [&](const Region& rg, const DAlloc& a, auto f) {
        for (u32 i0 = rg.clo[0] + (g + G - rg.clo[0] % G) % G; i0 < rg.chi[0]; i0 += G)
            for (u32 i1 = rg.clo[1]; i1 < rg.chi[1]; ++i1)
                for (u32 i2 = rg.clo[2]; i2 < rg.chi[2]; ++i2) f(alloc_local(a, i0, i1, i2));
    };
    for (u32 d = d0; d < nd; d += dstep) {
        if (nt() >= nd && d != d0) break;
        const u32 m = d + 2;
        // grouped reads: the device's kernels as one run of reader ids on
        // every cell of the shared region
        if (gmask && c.kdev_cnt[d]) {
            const u32 first = kern_first + c.kdev_base[d], nk = c.kdev_cnt[d];
            for (u32 j = 0; j < RD_CACHE; ++j) {
                if (!((gmask >> j) & 1)) continue;
                u32 kk = d * K;
                while (kk < (d + 1) * K && (c.k_rank[kk] == NONE || c.reg[kk * IG_MAX_ACCESS + j].empty)) ++kk;
                if (kk == (d + 1) * K) continue;
                const Region& rg = c.reg[kk * IG_MAX_ACCESS + j];
                const u32 al = live_containing(c, rg.buffer, m, rg.lo, rg.hi);
                if (!al) continue;
                const DAlloc& a = c.allocs[al];
                AmCell* cl = am_cells(c, a);
                own_cells(rg, a, [&](u32 l) {
                    if (nk == 1)
                        cell_add_reader_at(c, sh, m, cl + l, am_load(cl + l), first);
                    else
                        rd_append_range(c, sh, m, &cl[l].ov, first, nk);
                });
            }
        }
        for (u32 k = d * K; k < (d + 1) * K; ++k) {
            const u32 rk = c.k_rank[k];
            if (rk == NONE) continue;
            const u32 x = kern_first + c.kdev_base[d] + rk;
            for (u32 j = 0; j < A; ++j) {
                const Region& rg = c.reg[k * IG_MAX_ACCESS + j];
                if (rg.empty || !(rg.mode & IG_READ) || ((gmask >> j) & 1)) continue;
                const u32 al = live_containing(c, rg.buffer, m, rg.lo, rg.hi);
                if (!al) continue;
                const DAlloc& a = c.allocs[al];
                AmCell* cl = am_cells(c, a);
                own_cells(rg, a, [&](u32 l) {
                    const AmCell e = am_load(cl + l);
                    if ((e.w & ~W_ALLOC) == x) return;  // written by this kernel: no reader remains
                    cell_add_reader_at(c, sh, m, cl + l, e, x);
                });
            }
        }
    }
}

IGN void kernels_emit(DevCtx& c, Shared& sh, u32 kern_first) {
    if (uniform(sh.t_par))
        kernels_emit_par(c, sh, kern_first);
    else
        kernels_emit_seq(c, sh, kern_first);
}

// ===========================================================================
// Compile one task: allocation phase, coherence copies, kernels, edges.
// ===========================================================================
IGN void load_task(DevCtx& c, Shared& sh, u32 ci) {
    if (tid() == 0) {
        const DevCmd& cmd = c.cmds[ci];
        sh.t_cmd = ci;
        sh.t_id = cmd.arg;
        sh.t_dims = cmd.task.dims;
        sh.t_nacc = cmd.task.n_access;
        for (u32 d = 0; d < 3; ++d) {
            sh.t_lo[d] = cmd.task.box.min[d];
            sh.t_hi[d] = cmd.task.box.max[d];
        }
        // Writes through one_to_one, slice(d > 0) or a neighborhood without a
        // dim-0 radius stay inside their chunk's dim-0 range; chunks partition
        // that range, so such writes of different chunks cannot overlap.
        u32 stamps = 0;
        u64 wb = 0;
        for (u32 j = 0; j < cmd.task.n_access; ++j) {
            const ig_access& a = cmd.task.access[j];
            if (!(a.mode & IG_WRITE)) continue;
            wb |= 1ull << a.buffer;
            const bool confined = a.mapper == IG_MAP_ONE_TO_ONE || (a.mapper == IG_MAP_SLICE && a.slice_dim != 0) ||
                                  (a.mapper == IG_MAP_NEIGHBORHOOD && a.radius[0] == 0);
            if (!confined) stamps = 1;
        }
        sh.t_stamps = stamps;
        sh.t_wbufs = wb;
        // parallel kernel emission: every access to a written buffer stays in
        // its chunk's dim-0 range, and no pure read covers a region shared by
        // the chunks of a device (those share one scan in the ordered path)
        // A pure read of a buffer the task does not write through all,
        // fixed or slice(0) has the same region in every chunk; its cells
        // keep their writers through the task, so all kernels of a device
        // share one list of its sources (t_gmask), and the kernels stay
        // independent.  Beyond RD_CACHE such accesses use the ordered path.
        u32 par = 1, gmask = 0;
        for (u32 j = 0; j < cmd.task.n_access; ++j) {
            const ig_access& a = cmd.task.access[j];
            const bool confined = a.mapper == IG_MAP_ONE_TO_ONE || (a.mapper == IG_MAP_SLICE && a.slice_dim != 0) ||
                                  (a.mapper == IG_MAP_NEIGHBORHOOD && a.radius[0] == 0);
            const bool allish = a.mapper == IG_MAP_ALL || a.mapper == IG_MAP_FIXED ||
                                (a.mapper == IG_MAP_SLICE && a.slice_dim == 0);
            if (((wb >> a.buffer) & 1) && !confined) par = 0;
            if (a.mode == IG_READ && !((wb >> a.buffer) & 1) && allish) {
                if (j < RD_CACHE)
                    gmask |= 1u << j;
                else
                    par = 0;
            }
        }
        sh.t_par = par;
        sh.t_gmask = par ? gmask : 0;
    }
    bar();
}

// Every requirement of the task (regions in c.reg) lies in one live
// allocation of its memory: then the allocation phase has nothing to emit.
IGN bool regions_covered(DevCtx& c, Shared& sh) {
    const u32 A = sh.t_nacc, C = c.chunks;
    if (tid() == 0) sh.flag = 0;
    bar();
    for (u32 idx = tid(); idx < C * A; idx += nt()) {
        const u32 k = idx / A, j = idx % A;
        const Region& r = c.reg[k * IG_MAX_ACCESS + j];
        if (!r.empty && live_containing(c, r.buffer, mem_of_chunk(c, k), r.lo, r.hi) == 0) sh.flag = 1;
    }
    bar();
    return sh.flag == 0;
}

IGN void compile_task(DevCtx& c, Shared& sh, u32 ci, bool fresh) {
    tick(c, sh, PH_LOOKAHEAD);
    bool covered = fresh && sh.t_covered;
    if (!fresh) {
        load_task(c, sh, ci);
        compute_regions(c, sh);
        covered = regions_covered(c, sh);
    }
    if (tid() == 0) c.task_tc[sh.t_id] = ig_clock();
    unit_begin(c, sh);
    tick(c, sh, PH_COMPILE_REGIONS);
    if (!covered) {
        alloc_phase(c, sh);
        if (failed(sh)) return;
    } else if (tid() == 0) {
        sh.n_alloc_instr = 0;
    }
    tick(c, sh, PH_ALLOC);
    for (u32 i = tid(); i < c.n_mem; i += nt()) c.inbox_cnt[i] = 0;
    bar();
    coherence_count(c, sh);
    if (failed(sh)) return;
    coherence_big(c, sh);
    if (failed(sh)) return;
    tick(c, sh, PH_COH_COUNT);
    // scans: copies and kernels per device, inbox slots per memory
    for (u32 i = tid(); i < c.n_dev; i += nt()) {
        c.dev_base[i] = c.dev_cnt[i];
        c.kdev_base[i] = c.kdev_cnt[i];
    }
    for (u32 i = tid(); i < c.n_mem; i += nt()) c.inbox_off[i] = c.inbox_cnt[i];
    bar();
    const u32 n_copies = block_exscan(sh, c.dev_base, c.n_dev);
    const u32 n_kernels = block_exscan(sh, c.kdev_base, c.n_dev);
    block_exscan(sh, c.inbox_off, c.n_mem);
    for (u32 i = tid(); i < c.n_mem; i += nt()) c.inbox_cur[i] = c.inbox_off[i];
    const u32 n_task = sh.unit_n + n_copies + n_kernels;
    if (tid() == 0) {
        if ((u64)sh.unit_first + n_task > c.cap_instr) cap_error(sh, IG_CAP_INSTRUCTIONS);
        if (n_task > c.cap_unit) cap_error(sh, IG_CAP_UNIT);
        if (sh.s.n_binds + (u64)n_kernels * sh.t_nacc > c.cap_binds) cap_error(sh, IG_CAP_BINDINGS);
    }
    if (failed(sh)) return;
    const u32 copy_first = sh.unit_first + sh.unit_n;
    const u32 kern_first = copy_first + n_copies;
    tick(c, sh, PH_SCANS);
    coherence_emit(c, sh, copy_first);
    bar();
    tick(c, sh, PH_COH_EMIT);
    inbox_drain(c, sh);
    bar();
    tick(c, sh, PH_INBOX);
    kernels_emit(c, sh, kern_first);
    bar();
    tick(c, sh, PH_KERNELS);
    if (tid() == 0) sh.unit_n += n_copies + n_kernels;
    bar();
    unit_end(c, sh);
    if (tid() == 0) {
        sh.s.n_binds += (u64)n_kernels * sh.t_nacc;
        c.task_t1[sh.t_id] = ig_clock();
    }
    bar();
    tick(c, sh, PH_EDGES_OUT);
}

// ===========================================================================
// Lookahead (Sec. 4.3): command queue, allocating predicate, plans.
// ===========================================================================
IGD bool covered(DevCtx& c, Shared& sh, u32 b, u32 m, const i64 lo[3], const i64 hi[3]) {
    const u32 pi = b * c.n_mem + m;
    if (sh.s.qlen > 0 && c.plan_n[pi] != NONE) {
        const i64* p = c.plan + (size_t)pi * MAX_PLAN * 6;
        for (u32 i = 0; i < c.plan_n[pi]; ++i)
            if (box_contains(p + 6 * i, p + 6 * i + 3, lo, hi)) return true;
        return false;
    }
    return live_containing(c, b, m, lo, hi) != 0;
}

// allocating? (regions of the current task are in c.reg)
IGN bool task_allocating(DevCtx& c, Shared& sh) {
    const u32 A = sh.t_nacc, C = c.chunks;
    if (tid() == 0) sh.flag = 0;
    bar();
    for (u32 idx = tid(); idx < C * A; idx += nt()) {
        const u32 k = idx / A, j = idx % A;
        const Region& r = c.reg[k * IG_MAX_ACCESS + j];
        if (r.empty) continue;
        if (!covered(c, sh, r.buffer, mem_of_chunk(c, k), r.lo, r.hi)) sh.flag = 1;
    }
    bar();
    return sh.flag != 0;
}

IGN void plan_merge(DevCtx& c, Shared& sh) {
    const u32 A = sh.t_nacc, K = c.per_dev;
    for (u32 m = tid(); m < c.n_mem; m += nt()) {
        if (m < 2) continue;
        const u32 d = m - 2;
        i64* bx = c.wk_box + (size_t)tid() * c.cap_box * 6;
        for (u32 b = 0; b < sh.s.n_buffers; ++b) {
            bool any = false;
            for (u32 k = d * K; k < (d + 1) * K && !any; ++k)
                for (u32 j = 0; j < A; ++j) {
                    const Region& r = c.reg[k * IG_MAX_ACCESS + j];
                    if (!r.empty && r.buffer == b) any = true;
                }
            if (!any) continue;
            const u32 pi = b * c.n_mem + m;
            u32 n = 0;
            if (c.plan_n[pi] != NONE) {
                const i64* p = c.plan + (size_t)pi * MAX_PLAN * 6;
                for (u32 i = 0; i < c.plan_n[pi] * 6; ++i) bx[i] = p[i];
                n = c.plan_n[pi];
            } else {
                const u32 lb = pi * MAX_LIVE;
                for (u32 i = 0; i < c.live_n[pi]; ++i) {
                    const DAlloc& a = c.allocs[c.live[lb + i]];
                    for (u32 t = 0; t < 3; ++t) {
                        bx[6 * n + t] = a.lo[t];
                        bx[6 * n + 3 + t] = a.hi[t];
                    }
                    ++n;
                }
            }
            for (u32 k = d * K; k < (d + 1) * K; ++k)
                for (u32 j = 0; j < A; ++j) {
                    const Region& r = c.reg[k * IG_MAX_ACCESS + j];
                    if (r.empty || r.buffer != b) continue;
                    if (!box_push_merge(bx, n, c.cap_box, r.lo, r.hi)) {
                        cap_error(sh, IG_CAP_SCRATCH);
                        break;
                    }
                }
            n = merge_fixpoint(bx, n);
            if (n > MAX_PLAN) {
                cap_error(sh, IG_CAP_LIVE);
                continue;
            }
            i64* p = c.plan + (size_t)pi * MAX_PLAN * 6;
            for (u32 i = 0; i < n * 6; ++i) p[i] = bx[i];
            c.plan_n[pi] = n;
        }
    }
    bar();
}

// fresh: the regions of this task are still in c.reg (compiled right after intake)
IGN void compile_entry(DevCtx& c, Shared& sh, u32 entry, bool fresh) {
    if (entry & 0x80000000u) {
        compile_sync(c, sh, false);
    } else {
        compile_task(c, sh, entry, fresh);
    }
}

IGN void flush_queue(DevCtx& c, Shared& sh) {
    const u32 n = uniform(sh.s.qlen);
    for (u32 i = 0; i < n && !failed(sh); ++i) {
        if (tid() == 0) {
            sh.win_first = i + 1;
            sh.win_n = n - i - 1;
        }
        bar();
        compile_entry(c, sh, c.queue[i], false);
        bar();
    }
    const u32 NP = sh.s.n_buffers * c.n_mem;
    for (u32 i = tid(); i < NP; i += nt()) c.plan_n[i] = NONE;
    if (tid() == 0) {
        sh.s.qlen = 0;
        sh.s.h = 0;
        sh.win_n = 0;
    }
    bar();
}

IGN void push_command(DevCtx& c, Shared& sh, u32 entry, bool allocating) {
    const u32 qlen = uniform(sh.s.qlen);
    if (!c.lookahead || (qlen == 0 && !allocating)) {
        // compiled at once; without lookahead an allocating task still
        // compiles now, with its allocation phase
        if (tid() == 0) sh.win_n = 0;
        bar();
        compile_entry(c, sh, entry, !(entry & 0x80000000u));
        return;
    }
    if (allocating) plan_merge(c, sh);
    if (tid() == 0) {
        if (sh.s.qlen >= c.cap_queue) {
            cap_error(sh, IG_CAP_COMMANDS);
        } else {
            c.queue[sh.s.qlen++] = entry;
            if (allocating)
                sh.s.h = 0;
            else if (entry & 0x80000000u)
                sh.s.h += 1;
        }
    }
    if (failed(sh)) return;
    const bool full = sh.s.h >= c.flush_horizons || (c.queue_cap != 0 && sh.s.qlen >= c.queue_cap);
    bar();
    if (full) flush_queue(c, sh);
}

// ===========================================================================
// The task graph behind horizon mode 1 (Sec. 3.5): the critical-path length
// of an accepted task is one more than the longest of the sync point and
// the tasks it depends on.  Per buffer cell over the whole task's regions
// (every chunk; reads see the state before the task): a read depends on the
// last writer, a write on the readers since the last write, else on the
// last writer.  Lengths below the sync point's read as it (horizon and
// epoch compaction); a reader length at or below the latest epoch's is no
// reader.  Then reads raise the cells' reader length and writes set the
// writer length and clear the readers (a cell both read and written ends
// written).
// ===========================================================================
IGN void task_graph_step(DevCtx& c, Shared& sh) {
    const u32 A = sh.t_nacc, C = c.chunks;
    if (tid() == 0) sh.flag = sh.s.cp_sync;
    bar();
    const u32 cp_epoch = sh.s.cp_epoch;
    for (u32 idx = tid(); idx < C * A; idx += nt()) {
        const u32 k = idx / A, j = idx % A;
        const Region& r = c.reg[k * IG_MAX_ACCESS + j];
        if (r.empty) continue;
        const DBuf& B = c.bufs[r.buffer];
        const u32* wcp = W32(c, B.wcp_off);
        const u32* rcp = W32(c, B.rcp_off);
        u32 d = 0;
        for (u32 i0 = r.clo[0]; i0 < r.chi[0]; ++i0)
            for (u32 i1 = r.clo[1]; i1 < r.chi[1]; ++i1)
                for (u32 i2 = r.clo[2]; i2 < r.chi[2]; ++i2) {
                    const u32 cell = cell_of(B, i0, i1, i2);
                    const u32 w = wcp[cell], rd = rcp[cell];
                    if (r.mode & IG_READ) d = d > w ? d : w;
                    if (r.mode & IG_WRITE) {
                        const u32 x = rd > cp_epoch ? rd : w;
                        d = d > x ? d : x;
                    }
                }
        atomicMax(&sh.flag, d);
    }
    bar();
    const u32 cp = sh.flag + 1;
    for (u32 pass = 0; pass < 2; ++pass) {
        for (u32 idx = tid(); idx < C * A; idx += nt()) {
            const u32 k = idx / A, j = idx % A;
            const Region& r = c.reg[k * IG_MAX_ACCESS + j];
            if (r.empty || !(r.mode & (pass == 0 ? IG_READ : IG_WRITE))) continue;
            const DBuf& B = c.bufs[r.buffer];
            u32* wcp = W32(c, B.wcp_off);
            u32* rcp = W32(c, B.rcp_off);
            for (u32 i0 = r.clo[0]; i0 < r.chi[0]; ++i0)
                for (u32 i1 = r.clo[1]; i1 < r.chi[1]; ++i1)
                    for (u32 i2 = r.clo[2]; i2 < r.chi[2]; ++i2) {
                        const u32 cell = cell_of(B, i0, i1, i2);
                        if (pass == 0) {
                            atomicMax(&rcp[cell], cp);  // cp exceeds every length at or below the epoch's
                        } else {
                            wcp[cell] = cp;
                            rcp[cell] = 0;
                        }
                    }
        }
        bar();
    }
    if (tid() == 0) sh.s.cp_max = sh.s.cp_max > cp ? sh.s.cp_max : cp;
    bar();
}

// ===========================================================================
// Command intake
// ===========================================================================
IGN void intake_task(DevCtx& c, Shared& sh, u32 ci) {
    load_task(c, sh, ci);
    if (tid() == 0) c.task_t0[sh.t_id] = ig_clock();
    tick(c, sh, PH_OTHER);
    if (tid() == 0) *c.miss_n = 0;
    bar();
    compute_regions(c, sh);
    if (uniform(*c.miss_n)) {
        refine_all(c, sh);
        if (failed(sh)) return;
        compute_regions(c, sh);
        if (uniform(*c.miss_n) && tid() == 0) set_error(sh, IG_E_INTERNAL);
        if (failed(sh)) return;
    }
    tick(c, sh, PH_INTAKE_REGIONS);
    // Sec. 4.4 checks
    const u32 A = sh.t_nacc, C = c.chunks, t = sh.t_id;
    if (tid() == 0) {
        sh.flag = 0;
        sh.flag2 = 0;
    }
    bar();
    for (u32 idx = tid(); idx < C * A; idx += nt()) {
        const u32 k = idx / A, j = idx % A;
        const Region& r = c.reg[k * IG_MAX_ACCESS + j];
        if (r.empty) continue;
        const DBuf& B = c.bufs[r.buffer];
        const bool check_read = (r.mode & IG_READ) && B.uninit != 0;
        const bool check_write = (r.mode & IG_WRITE) && sh.t_stamps;
        if (!check_read && !check_write) continue;
        u64* stamp = W64(c, B.stamp_off);
        const u32* init = W32(c, B.init_off);
        const u64 mine = ((u64)(t + 1) << 32) | k;
        for (u32 i0 = r.clo[0]; i0 < r.chi[0]; ++i0)
            for (u32 i1 = r.clo[1]; i1 < r.chi[1]; ++i1)
                for (u32 i2 = r.clo[2]; i2 < r.chi[2]; ++i2) {
                    const u32 cell = cell_of(B, i0, i1, i2);
                    if (check_read && !init[cell]) sh.flag2 = 1;
                    if (check_write) {
                        u64 old = stamp[cell];
                        while (true) {
                            if ((old >> 32) == (u64)(t + 1)) {
                                if (old != mine) sh.flag = 1;
                                break;
                            }
                            const u64 seen = atomicCAS((unsigned long long*)&stamp[cell], (unsigned long long)old,
                                                       (unsigned long long)mine);
                            if (seen == old) break;
                            old = seen;
                        }
                    }
                }
    }
    const bool overlap = uniform(sh.flag) != 0;
    if (tid() == 0) {
        const i32 st = overlap ? IG_E_OVERLAPPING_WRITE : (sh.flag2 ? IG_W_UNINIT_READ : IG_OK);
        c.task_status[sh.s.n_tasks] = st;
        sh.s.n_tasks += 1;
        if (overlap) {
            sh.s.rejected += 1;
            const u64 now = ig_clock();
            c.task_tq[sh.t_id] = now;
            c.task_tc[sh.t_id] = now;
            c.task_t1[sh.t_id] = now;
        }
        if (st == IG_W_UNINIT_READ) sh.s.warnings += 1;
    }
    bar();
    if (overlap) return;
    for (u32 idx = tid(); idx < C * A; idx += nt()) {
        const u32 k = idx / A, j = idx % A;
        const Region& r = c.reg[k * IG_MAX_ACCESS + j];
        if (r.empty || !(r.mode & IG_WRITE)) continue;
        DBuf& B = c.bufs[r.buffer];
        if (B.uninit == 0) continue;
        u32* init = W32(c, B.init_off);
        for (u32 i0 = r.clo[0]; i0 < r.chi[0]; ++i0)
            for (u32 i1 = r.clo[1]; i1 < r.chi[1]; ++i1)
                for (u32 i2 = r.clo[2]; i2 < r.chi[2]; ++i2)
                    if (atomicExch(&init[cell_of(B, i0, i1, i2)], 1u) == 0) atomicAdd(&B.uninit, 0xFFFFFFFFu);
    }
    bar();
    if (c.horizon_mode == 1) task_graph_step(c, sh);
    tick(c, sh, PH_INTAKE_CHECKS);
    const bool allocating = task_allocating(c, sh);
    if (tid() == 0) sh.t_covered = (sh.s.qlen == 0 && !allocating) ? 1u : 0u;
    bar();
    tick(c, sh, PH_LOOKAHEAD);
    if (tid() == 0) c.task_tq[sh.t_id] = ig_clock();
    push_command(c, sh, ci, allocating);
    if (failed(sh)) return;
    if (tid() == 0) {
        sh.s.tasks_since_sync += 1;
        sh.do_horizon = 0;
        if (c.horizon_mode == 1) {
            // Sec. 3.5 from the task graph: the path grew by horizon_step
            // since the last horizon or epoch, or enough tasks came since
            if (sh.s.cp_max - sh.s.cp_last >= c.horizon_step || sh.s.tasks_since_sync >= c.horizon_max_tasks) {
                if (sh.s.cp_pending) sh.s.cp_sync = sh.s.cp_pending;
                sh.s.cp_pending = sh.s.cp_max + 1;
                sh.s.cp_last = sh.s.cp_max;
                sh.s.tasks_since_sync = 0;
                sh.do_horizon = 1;
            }
        } else if (sh.s.tasks_since_sync == c.horizon_step) {
            sh.s.tasks_since_sync = 0;
            sh.do_horizon = 1;
        }
    }
    if (uniform(sh.do_horizon)) push_command(c, sh, 0x80000000u, false);
}

IGN void create_buffer(DevCtx& c, Shared& sh, const DevCmd& cmd) {
    if (tid() == 0) {
        const u32 b = sh.s.n_buffers;
        if (b >= MAX_BUF) {
            cap_error(sh, IG_CAP_BUFFERS);
        } else {
            DBuf& B = c.bufs[b];
            B.alive = 1;
            B.dims = cmd.dims;
            B.init = cmd.init;
            B.user_alloc = 0;
            for (u32 d = 0; d < 3; ++d) {
                B.ext[d] = cmd.ext[d];
                B.n[d] = 1;
                B.bp_off[d] = heap_alloc(c, sh, 4);
                if (B.bp_off[d]) {
                    WI64(c, B.bp_off[d])[0] = 0;
                    WI64(c, B.bp_off[d])[1] = cmd.ext[d];
                }
            }
            for (u32 d = 0; d < 3; ++d) {
                B.hx_off[d] = 0;
                if (B.bp_off[d]) hx_build(c, sh, B, d);
            }
            B.ncells = 1;
            B.prod_off = heap_alloc(c, sh, 1);
            B.pm_off = heap_alloc(c, sh, 1);
            B.mask_off = heap_alloc(c, sh, 2 * c.mw);
            B.init_off = heap_alloc(c, sh, 1);
            B.stamp_off = heap_alloc(c, sh, 2);
            B.wcp_off = heap_alloc(c, sh, 1);
            B.rcp_off = heap_alloc(c, sh, 1);
            if (!sh.s.error) {
                W32(c, B.wcp_off)[0] = 0;
                W32(c, B.rcp_off)[0] = 0;
                W32(c, B.prod_off)[0] = cmd.init ? sh.s.S : NONE;
                W32(c, B.pm_off)[0] = cmd.init ? 0 : NONE;
                for (u32 w = 0; w < c.mw; ++w) W64(c, B.mask_off)[w] = (cmd.init && w == 0) ? 1ull : 0ull;
                W32(c, B.init_off)[0] = cmd.init ? 1 : 0;
                B.uninit = cmd.init ? 0 : 1;
                W64(c, B.stamp_off)[0] = 0;
                for (u32 m = 0; m < c.n_mem; ++m) {
                    c.live_n[b * c.n_mem + m] = 0;
                    c.plan_n[b * c.n_mem + m] = NONE;
                }
                if (cmd.init) {
                    // host data lives in user memory M0, produced before the current sync point
                    const u32 id = sh.s.next_alloc++;
                    if (id >= c.cap_allocs) {
                        cap_error(sh, IG_CAP_ALLOCS);
                    } else {
                        DAlloc& a = c.allocs[id];
                        a.buffer = b;
                        a.mem = 0;
                        a.alive = 1;
                        a.ncells = 1;
                        for (u32 d = 0; d < 3; ++d) {
                            a.lo[d] = 0;
                            a.hi[d] = cmd.ext[d];
                            a.clo[d] = 0;
                            a.chi[d] = 1;
                        }
                        a.am_off = heap_alloc(c, sh, 4);
                        if (!sh.s.error) cell_init(am_cells(c, a), sh.s.S);
                        c.live[(b * c.n_mem + 0) * MAX_LIVE] = id;
                        c.live_n[b * c.n_mem + 0] = 1;
                        B.user_alloc = id;
                    }
                }
                sh.s.n_buffers = b + 1;
            }
        }
    }
    bar();
}

// Sec. 3.2: a destroyed buffer's device allocations are freed (ascending id)
// Mark the LIFETIME sources one allocation-map cell gives a FREE (its writer
// and readers after substitution) in a bitmap over ids [S, S + R); with
// `shared` the bitmap is marked by several threads at once.
IGD void free_mark_cell(DevCtx& c, Shared& sh, const AmCell& e, u32 R, u64* bm, bool shared) {
    const u32 S = sh.s.S, E = sh.s.E;
    auto mark = [&](u32 id) {
        const u32 o = id - S;
        if (o >= R) {
            set_error(sh, IG_E_INTERNAL);
            return;
        }
        if (shared)
            atomicOr(&bm[o >> 6], 1ull << (o & 63));
        else
            bm[o >> 6] |= 1ull << (o & 63);
    };
    const u32 wr = e.w & ~W_ALLOC;
    mark(wr < S ? S : wr);
    u32 r;
    if (e.r0 != NONE && eff_r(sh, e.r0, r)) mark(r);
    if (e.r1 != NONE && eff_r(sh, e.r1, r)) mark(r);
    rd_each(c, e.ov, [&](u32 first, u32 n) {
        const u32 end = first + n;
        u32 lo = first < E ? E : first;
        if (lo >= end) return;
        if (lo < S) {
            mark(S);
            lo = S;
        }
        if (lo >= end) return;  // the whole run reads as S
        if (end - S > R) {
            set_error(sh, IG_E_INTERNAL);
            return;
        }
        // bits [lo - S, end - S), word by word
        for (u32 o = lo - S; o < end - S;) {
            const u32 wd = o >> 6, b0 = o & 63;
            const u32 b1 = (end - S) - (wd << 6) < 64 ? (end - S) - (wd << 6) : 64;
            const u64 mk = (b1 == 64 ? ~0ull : ((1ull << b1) - 1)) & ~((1ull << b0) - 1);
            if (shared)
                atomicOr(&bm[wd], mk);
            else
                bm[wd] |= mk;
            o = (wd << 6) + b1;
        }
    });
}

// FREE x of allocation a by one thread (the allocation phase): its sources
// from a bitmap over [S, x) in the thread's scratch, staged in id order;
// a range beyond the bitmap's size uses a sorted source list instead.
IGN void free_stage_one(DevCtx& c, Shared& sh, u32 x, const DAlloc& a, u64* bm) {
    const u32 S = sh.s.S, R = x - S;
    if ((u64)R > 64ull * c.cap_scr) {
        SrcSet s;
        ss_init(c, s);
        free_edges(c, sh, s, a);
        stage(c, sh, x, s);
        return;
    }
    const u32 words = (R + 63) / 64;
    for (u32 i = 0; i < words; ++i) bm[i] = 0;
    const AmCell* cl = am_cells(c, a);
    for (u32 l = 0; l < a.ncells; ++l) free_mark_cell(c, sh, am_load(cl + l), R, bm, false);
    u32 n = 0;
    for (u32 i = 0; i < words; ++i) n += __popcll(bm[i]);
    const u32 slot = x - sh.unit_first;
    const u32 cnt = n ? n : 1;
    const u32 off = atomicAdd(&sh.stage_top, cnt);
    if ((u64)off + cnt > (u64)c.cap_unit * 8 || slot >= c.cap_unit) {
        cap_error(sh, IG_CAP_UNIT);
        return;
    }
    c.tab_off[slot] = off;
    c.tab_cnt[slot] = cnt;
    if (n == 0) {  // no dependency: wait for the synchronisation point
        c.stage_from[off] = S;
        c.stage_kind[off] = IG_DEP_SYNC;
        c.has_succ[S] = 1;
        return;
    }
    u32 o = off;
    for (u32 i = 0; i < words; ++i) {
        u64 v = bm[i];
        while (v) {
            const u32 bit = __ffsll((long long)v) - 1;
            v &= v - 1;
            const u32 from = S + (i << 6) + bit;
            c.stage_from[o] = from;
            c.stage_kind[o] = IG_DEP_LIFETIME;
            c.has_succ[from] = 1;
            ++o;
        }
    }
}

// The FREE x of allocation a (Sec. 3.2), its edges found by the team of its
// memory: every writer and reader of the allocation, after substitution,
// lies in [S, x), so the members mark them in a bitmap of that range (one
// part of the cells each) and the set bits, in order, are the sorted,
// duplicate-free LIFETIME sources.  A range beyond the bitmap's size takes
// the member-0 path with a sorted source list.
IGN void team_free(DevCtx& c, Shared& sh, bool act, u32 m, u32 g, u32 G, u32 ai, u32 x) {
    const u32 S = sh.s.S, E = sh.s.E;
    const u32 R = act ? x - S : 0;
    const u32 w = m % nt();
    IG_SIM_CHECK(!act || w < c.n_workers, "free bitmap per worker");
    u64* bm = c.wk_key + (size_t)w * c.cap_scr;
    u32* tm = c.tm + 4 * (size_t)m;
    const bool bits = act && (u64)R <= 64ull * c.cap_scr;
    const DAlloc& a = c.allocs[act ? ai : 0];
    const u32 words = (R + 63) / 64;
    if (act && g == 0) put_instr(c, x, IG_FREE, 0, NONE, NONE, a.buffer, m, 0xFFFF, ai, 0, a.lo, a.hi);
    if (act && !bits && g == 0) {
        SrcSet s;
        ss_init(c, s);
        free_edges(c, sh, s, a);
        stage(c, sh, x, s);
    }
    if (bits)
        for (u32 i = g; i < words; i += G) bm[i] = 0;
    bar();
    const u32 per = act ? (a.ncells + G - 1) / G : 0;
    const u32 l0 = act && g * per < a.ncells ? g * per : (act ? a.ncells : 0);
    const u32 l1 = act && l0 + per < a.ncells ? l0 + per : (act ? a.ncells : 0);
    if (bits) {
        const AmCell* cl = am_cells(c, a);
        for (u32 l = l0; l < l1; ++l) free_mark_cell(c, sh, am_load(cl + l), R, bm, true);
    }
    bar();
    // set bits -> staged edges, in order
    const u32 wpg = (words + G - 1) / G;
    const u32 w0 = bits && g * wpg < words ? g * wpg : words, w1 = bits && w0 + wpg < words ? w0 + wpg : words;
    u32 cnt = 0;
    if (bits)
        for (u32 i = w0; i < w1; ++i) cnt += __popcll(bm[i]);
    u32 tot;
    const u32 excl = block_excl(sh, bits ? cnt : 0, &tot);
    if (bits && g == 0) tm[0] = excl;
    bar();
    const u32 off = bits ? excl - tm[0] : 0;
    if (bits && g == G - 1) tm[1] = off + cnt;
    bar();
    if (bits && g == 0) {
        const u32 n = tm[1] ? tm[1] : 1;
        const u32 slot = x - sh.unit_first;
        const u32 at = atomicAdd(&sh.stage_top, n);
        if ((u64)at + n > (u64)c.cap_unit * 8 || slot >= c.cap_unit) {
            cap_error(sh, IG_CAP_UNIT);
        } else {
            c.tab_off[slot] = at;
            c.tab_cnt[slot] = n;
            if (tm[1] == 0) {  // no dependency: wait for the synchronisation point
                c.stage_from[at] = S;
                c.stage_kind[at] = IG_DEP_SYNC;
                c.has_succ[S] = 1;
            }
        }
        tm[2] = at;
    }
    if (failed(sh)) return;
    if (bits && cnt) {
        u32 o = tm[2] + off;
        for (u32 i = w0; i < w1; ++i) {
            u64 v = bm[i];
            while (v) {
                const u32 bit = __ffsll((long long)v) - 1;
                v &= v - 1;
                const u32 from = S + (i << 6) + bit;
                c.stage_from[o] = from;
                c.stage_kind[o] = IG_DEP_LIFETIME;
                c.has_succ[from] = 1;
                ++o;
            }
        }
    }
    // the allocation's reader blocks go back to the memory's free list
    if (act) {
        AmCell* cl = am_cells(c, a);
        for (u32 l = l0; l < l1; ++l)
            if (cl[l].ov) rd_clear(c, m, &cl[l].ov);
    }
    bar();
}

IGN void destroy_buffer(DevCtx& c, Shared& sh, u32 b) {
    unit_begin(c, sh);
    if (tid() == 0) {
        u32 n = 0, most = 0;
        for (u32 m = 2; m < c.n_mem; ++m) {
            const u32 lb = (b * c.n_mem + m) * MAX_LIVE;
            for (u32 i = 0; i < c.live_n[b * c.n_mem + m]; ++i) c.cons_off[n++] = c.live[lb + i];
            most = c.live_n[b * c.n_mem + m] > most ? c.live_n[b * c.n_mem + m] : most;
        }
        sh.flag2 = most;
        for (u32 i = 1; i < n; ++i)
            for (u32 j = i; j > 0 && c.cons_off[j] < c.cons_off[j - 1]; --j) {
                const u32 v = c.cons_off[j];
                c.cons_off[j] = c.cons_off[j - 1];
                c.cons_off[j - 1] = v;
            }
        if ((u64)sh.unit_first + n > c.cap_instr) cap_error(sh, IG_CAP_INSTRUCTIONS);
        if (n > c.cap_unit) cap_error(sh, IG_CAP_UNIT);
        sh.unit_n = n;
    }
    if (failed(sh)) return;
    const u32 n = sh.unit_n, rounds = sh.flag2;
    // round r: every memory's r-th FREE (ascending id), by the memory's team
    const u32 G = team_size(c), TP = nt() / G, ts = tid() / G, g = tid() % G;
    for (u32 rnd = 0; rnd < rounds; ++rnd)
        for (u32 base = 0; base < c.n_dev; base += TP) {
            const u32 m = base + ts + 2;
            u32 i = 0, seen = 0;
            bool act = false;
            if (m < c.n_mem)
                for (; i < n; ++i)
                    if (c.allocs[c.cons_off[i]].mem == m && seen++ == rnd) {
                        act = true;
                        break;
                    }
            team_free(c, sh, act, m, g, G, act ? c.cons_off[i] : 0, sh.unit_first + i);
            if (failed(sh)) return;
        }
    unit_end(c, sh);
    if (tid() == 0) {
        DBuf& B = c.bufs[b];
        for (u32 i = 0; i < n; ++i) {
            DAlloc& a = c.allocs[c.cons_off[i]];
            a.alive = 0;
            heap_release(c, a.am_off);
        }
        for (u32 m = 0; m < c.n_mem; ++m) c.live_n[b * c.n_mem + m] = 0;
        B.alive = 0;
    }
    bar();
    // the user allocation's reader lists go back to M0's free list
    if (c.bufs[b].user_alloc && owner_of(0) == tid()) release_readers(c, c.allocs[c.bufs[b].user_alloc]);
    bar();
    if (tid() == 0) {
        DBuf& B = c.bufs[b];
        if (B.user_alloc) {
            DAlloc& ua = c.allocs[B.user_alloc];
            ua.alive = 0;
            heap_release(c, ua.am_off);
        }
        for (u32 d = 0; d < 3; ++d) {
            heap_release(c, B.bp_off[d]);
            heap_release(c, B.hx_off[d]);
        }
        heap_release(c, B.prod_off);
        heap_release(c, B.pm_off);
        heap_release(c, B.mask_off);
        heap_release(c, B.init_off);
        heap_release(c, B.stamp_off);
        heap_release(c, B.wcp_off);
        heap_release(c, B.rcp_off);
    }
    bar();
}

IGN void init_state(DevCtx& c, Shared& sh) {
    // I0, the initial epoch, and empty tables
    for (u32 i = tid(); i < 32; i += nt()) c.heap_free[i] = 0;
    for (u32 i = tid(); i < c.n_mem; i += nt()) c.rb_free[i] = 0ull;
    if (tid() == 0) {
        Scalars& s = sh.s;
        s.n_instr = 1;
        s.n_edges = 0;
        s.n_binds = 0;
        s.warnings = s.rejected = s.resizes = 0;
        s.cmd_next = 0;
        s.n_tasks = 0;
        s.next_alloc = 1;
        s.S = 0;
        s.E = 0;
        s.pending = NONE;
        s.last_sync = 0;
        s.tasks_since_sync = 0;
        s.h = 0;
        s.qlen = 0;
        s.n_buffers = 0;
        s.finished = 0;
        s.heap_top = 16;
        s.rb_top = 1;
        s.error = 0;
        const i64 z[3] = {0, 0, 0};
        put_instr(c, 0, IG_EPOCH, 0, NONE, NONE, NONE, 0xFFFF, 0xFFFF, 0, 0, z, z);
    }
    bar();
}

// Tasks are compiled in id order; those before the first task still held in
// the lookahead queue have all their records.
IGD u32 done_prefix(const DevCtx& c, const Scalars& s) {
    for (u32 i = 0; i < s.qlen; ++i) {
        const u32 e = c.queue[i];
        if (!(e & 0x80000000u)) return c.cmds[e].arg;
    }
    return s.n_tasks;
}

// Analyse the uploaded commands from the context's position on; window > 0
// stops after that many commands (the rest follows in later launches).
// An epoch follows everything in the task graph so far (thread 0).
IGD void epoch_task_graph(Shared& sh) {
    const u32 e = sh.s.cp_max + 1;
    sh.s.cp_epoch = sh.s.cp_sync = sh.s.cp_max = sh.s.cp_last = e;
    sh.s.cp_pending = 0;
}

IGN void analyse(DevCtx& c, Shared& sh, u32 window) {
    if (tid() == 0) {
        sh.s = c.s;
        sh.tick = ig_clock();
    }
    sh.rbs_head[tid()] = 0;
    bar();
    const u32 first = sh.s.cmd_next;
    const u32 end = window && c.cmd_end - first > window ? first + window : c.cmd_end;
    if (uniform(sh.s.cmd_next == 0 && sh.s.n_instr == 0)) init_state(c, sh);
    while (true) {
        const u32 ci = sh.s.cmd_next;
        const bool go = ci < end && sh.s.error == 0;
        bar();
        if (!go) break;
        const DevCmd& cmd = c.cmds[ci];
        switch (cmd.kind) {
            case CMD_BUFFER:
                create_buffer(c, sh, cmd);
                break;
            case CMD_TASK:
                intake_task(c, sh, ci);
                break;
            case CMD_EPOCH:
                flush_queue(c, sh);
                if (tid() == 0) {
                    sh.s.tasks_since_sync = 0;
                    epoch_task_graph(sh);
                }
                bar();
                compile_sync(c, sh, true);
                break;
            case CMD_DESTROY:
                flush_queue(c, sh);
                destroy_buffer(c, sh, cmd.arg);
                break;
            case CMD_SHUTDOWN: {
                flush_queue(c, sh);
                const u32 nb = uniform(sh.s.n_buffers);
                for (u32 b = 0; b < nb && !failed(sh); ++b)
                    if (uniform(c.bufs[b].alive)) destroy_buffer(c, sh, b);
                if (tid() == 0) {
                    sh.s.tasks_since_sync = 0;
                    epoch_task_graph(sh);
                }
                bar();
                compile_sync(c, sh, true);
                if (tid() == 0) sh.s.finished = 1;
                break;
            }
            default:
                if (tid() == 0) set_error(sh, IG_E_INVALID);
        }
        bar();
        if (tid() == 0 && !sh.s.error) sh.s.cmd_next = ci + 1;
        bar();
    }
    rb_stash_return(c, sh);
    bar();
    if (tid() == 0) {
        sh.s.done_tasks = done_prefix(c, sh.s);
        c.s = sh.s;
    }
}

// Forget all analysis results of one context (block-wide).
IGD void reset_state(DevCtx& c, u32 t, u32 n) {
    u32* w = (u32*)&c.s;
    for (u32 i = t; i < sizeof(Scalars) / 4; i += n) w[i] = 0;
    for (u32 i = t; i < 32; i += n) c.phase[i] = 0;
}

// Progress of one context: done tasks, seen tasks, error, finished.
IGD void gather_progress(const DevCtx& c, u64* out) {
    out[0] = c.s.done_tasks | ((u64)c.s.n_tasks << 32);
    out[1] = (u64)(u32)c.s.error | ((u64)c.s.cap_what << 32);
    out[2] = c.s.finished;
    out[3] = c.s.cmd_next;
}

// ===========================================================================
// Record digests and statistics (parallel over records)
// ===========================================================================
IGD u64 splitmix64(u64 x) {
    u64 z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

IGD u64 fnv_words(const u64* w, u32 n) {
    u64 h = 0xcbf29ce484222325ull;
    for (u32 i = 0; i < n; ++i)
        for (u32 b = 0; b < 8; ++b) {
            h ^= (w[i] >> (8 * b)) & 0xFF;
            h *= 0x100000001b3ull;
        }
    return h;
}

IGD u64 w32(u32 v) { return v; }
IGD u64 w16(u16 v) { return v; }

IGD void instr_words(const DevCtx& c, u64 i, u64 w[12]) {
    w[0] = i;
    w[1] = (u64)c.i_kind[i] | ((u64)c.i_flags[i] << 8) | ((u64)c.i_mem[i] << 16) | ((u64)c.i_src_mem[i] << 32);
    w[2] = (u64)c.i_task[i] | ((u64)c.i_chunk[i] << 32);
    w[3] = c.i_buffer[i];
    w[4] = c.i_alloc[i];
    w[5] = c.i_src_alloc[i];
    for (u32 d = 0; d < 6; ++d) w[6 + d] = (u64)c.i_box[d * c.cap_instr + i];
}

}  // namespace igd

using namespace igd;

// ===========================================================================
// Kernels
// ===========================================================================
#ifndef IG_HOST_SIM
// The analysis kernel is compiled twice: here for workgroups of up to 256
// threads (a register budget of up to 512 per lane, so the per-worker source
// sets and cell records stay in registers), and in ig_kernels_wide.hip for up
// to 1024 threads (128 registers per lane).
#ifdef IG_WIDE_ONLY
__global__ void __launch_bounds__(1024) ig_analyse_wide(DevCtx* const* ctxs, u32 window) {
    __shared__ Shared sh;
    analyse(*ctxs[blockIdx.x], sh, window);
}

namespace igrt {
int launch_analyse_wide(DevCtx* const* ptrs, unsigned n_blocks, unsigned threads, unsigned window, void* stream) {
    hipLaunchKernelGGL(ig_analyse_wide, dim3(n_blocks), dim3(threads), 0, (hipStream_t)stream, ptrs, window);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
}  // namespace igrt
#else
__global__ void __launch_bounds__(256) ig_analyse(DevCtx* const* ctxs, u32 window) {
    __shared__ Shared sh;
    analyse(*ctxs[blockIdx.x], sh, window);
}

__global__ void __launch_bounds__(64) ig_reset(DevCtx* const* ctxs) {
    reset_state(*ctxs[blockIdx.x], threadIdx.x, blockDim.x);
}

__global__ void __launch_bounds__(256) ig_gather(DevCtx* const* ctxs, u32 n, u64* out) {
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) gather_progress(*ctxs[i], out + 4 * (size_t)i);
}

__global__ void ig_pack_instructions(const DevCtx* c, u64 first, u64 n, ig_instruction* out) {
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 x = first + i;
    ig_instruction r;
    r.id = x;
    r.kind = c->i_kind[x];
    r.flags = c->i_flags[x];
    r.mem = c->i_mem[x];
    r.src_mem = c->i_src_mem[x];
    r.pad0 = 0;
    r.task = c->i_task[x];
    r.chunk = c->i_chunk[x];
    r.buffer = c->i_buffer[x];
    r.pad1 = 0;
    r.alloc = c->i_alloc[x];
    r.src_alloc = c->i_src_alloc[x];
    for (u32 d = 0; d < 3; ++d) {
        r.box.min[d] = c->i_box[d * c->cap_instr + x];
        r.box.max[d] = c->i_box[(3 + d) * c->cap_instr + x];
    }
    out[i] = r;
}

__global__ void ig_pack_bindings(const DevCtx* c, u64 first, u64 n, ig_binding* out) {
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ig_binding r;
    r.instr = c->b_instr[first + i];
    r.access = c->b_access[first + i];
    r.pad = 0;
    r.alloc = c->b_alloc[first + i];
    out[i] = r;
}

__global__ void ig_pack_edges(const DevCtx* c, u64 first, u64 n, ig_edge* out) {
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ig_edge r;
    r.from = c->e_from[first + i];
    r.to = c->e_to[first + i];
    r.kinds = c->e_kinds[first + i];
    r.pad = 0;
    out[i] = r;
}

__global__ void __launch_bounds__(256) ig_stats_kernel(const DevCtx* c, u64 ni, u64 nb, u64 ne, DevStats* out) {
    __shared__ unsigned long long acc[3 + 8 + 5];
    if (threadIdx.x < 16) acc[threadIdx.x] = 0;
    __syncthreads();
    const u64 stride = (u64)gridDim.x * blockDim.x;
    unsigned long long dig[3] = {0, 0, 0};
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < ni; i += stride) {
        u64 w[12];
        instr_words(*c, i, w);
        dig[0] += splitmix64(fnv_words(w, 12) ^ splitmix64(i));
        atomicAdd(&acc[3 + (c->i_kind[i] & 7)], 1ull);
    }
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += stride) {
        u64 w[3] = {c->b_instr[i], c->b_access[i], c->b_alloc[i]};
        dig[1] += splitmix64(fnv_words(w, 3) ^ splitmix64(i));
    }
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += stride) {
        u64 w[3] = {c->e_from[i], c->e_to[i], c->e_kinds[i]};
        dig[2] += splitmix64(fnv_words(w, 3) ^ splitmix64(i));
        const u32 k = c->e_kinds[i];
        for (u32 b = 0; b < 5; ++b)
            if (k & (1u << b)) atomicAdd(&acc[11 + b], 1ull);
    }
    for (u32 q = 0; q < 3; ++q) atomicAdd(&acc[q], dig[q]);
    __syncthreads();
    if (threadIdx.x < 16) {
        unsigned long long* dst = threadIdx.x < 3 ? &out->digest[threadIdx.x]
                                  : threadIdx.x < 11 ? &out->per_kind[threadIdx.x - 3]
                                                     : &out->per_dep[threadIdx.x - 11];
        atomicAdd(dst, acc[threadIdx.x]);
    }
}

// Fixed device memory of the entry points that allocate nothing
// (ig_batch_progress_noalloc): a context-pointer table followed by the
// gathered progress words.  Every GPU holds its own copy until the process
// ends.  Host code must never pass this name to a kernel or a copy (on the
// host it is only a stand-in): it uses the device address that
// igrt::noalloc_scratch looks up per device.
static __device__ __align__(256) unsigned char scratch[IG_NOALLOC_SCRATCH_BYTES];

namespace igrt {
static thread_local char g_err[256];
static int check(hipError_t e) {
    if (e != hipSuccess) {
        snprintf(g_err, sizeof g_err, "%s", hipGetErrorString(e));
        return -1;
    }
    return 0;
}
const char* last_error() { return g_err; }
int dev_malloc(void** p, size_t bytes) { return check(hipMalloc(p, bytes)); }
int dev_free(void* p) { return check(hipFree(p)); }
int host_malloc_pinned(void** p, size_t bytes) { return check(hipHostMalloc(p, bytes, hipHostMallocDefault)); }
int host_free_pinned(void* p) { return check(hipHostFree(p)); }
int copy_h2d(void* dst, const void* src, size_t bytes, void* stream) {
    return check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, (hipStream_t)stream));
}
int copy_d2h(void* dst, const void* src, size_t bytes, void* stream) {
    return check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream));
}
int memset_d(void* dst, int v, size_t bytes, void* stream) {
    return check(hipMemsetAsync(dst, v, bytes, (hipStream_t)stream));
}
int stream_sync(void* stream) { return check(hipStreamSynchronize((hipStream_t)stream)); }
double clock_khz() {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return (double)khz;
}
int launch_analyse(DevCtx* const* ptrs, unsigned n_blocks, unsigned threads, unsigned window, void* stream) {
    if (threads > 256) {
        if (launch_analyse_wide(ptrs, n_blocks, threads, window, stream) != 0) return check(hipGetLastError());
        return 0;
    }
    hipLaunchKernelGGL(ig_analyse, dim3(n_blocks), dim3(threads), 0, (hipStream_t)stream, ptrs, window);
    return check(hipGetLastError());
}
static unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }
int launch_reset(DevCtx* const* ptrs, unsigned n, void* stream) {
    if (!n) return 0;
    hipLaunchKernelGGL(ig_reset, dim3(n), dim3(64), 0, (hipStream_t)stream, ptrs);
    return check(hipGetLastError());
}
int launch_gather(DevCtx* const* ptrs, unsigned n, uint64_t* out, void* stream) {
    if (!n) return 0;
    hipLaunchKernelGGL(ig_gather, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, ptrs, n,
                       (u64*)out);
    return check(hipGetLastError());
}
// The graph is captured on a stream of its own (default priority) and
// launched on the caller's stream.
int graph_capture(DevCtx* const* ptrs, unsigned n, unsigned threads, void* stream, void** exec) {
    (void)stream;
    hipStream_t cs;
    if (check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking))) return -1;
    hipGraph_t g = nullptr;
    int rc = check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    if (!rc) rc = launch_reset(ptrs, n, cs);
    if (!rc) rc = launch_analyse(ptrs, n, threads, 0, cs);
    const int rc_end = check(hipStreamEndCapture(cs, &g));
    if (!rc) rc = rc_end;
    hipGraphExec_t e = nullptr;
    if (!rc) rc = check(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (rc) return rc;
    *exec = (void*)e;
    return 0;
}
int graph_launch(void* exec, void* stream) {
    return check(hipGraphLaunch((hipGraphExec_t)exec, (hipStream_t)stream));
}
int graph_destroy(void* exec) { return check(hipGraphExecDestroy((hipGraphExec_t)exec)); }
int event_create(void** ev) {
    hipEvent_t e = nullptr;
    if (check(hipEventCreateWithFlags(&e, hipEventDisableTiming))) return -1;
    *ev = (void*)e;
    return 0;
}
int event_record(void* ev, void* stream) { return check(hipEventRecord((hipEvent_t)ev, (hipStream_t)stream)); }
int event_query(void* ev) {
    const hipError_t e = hipEventQuery((hipEvent_t)ev);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) {
        (void)hipGetLastError();
        return 0;
    }
    check(e);
    return -1;
}
int event_sync(void* ev) { return check(hipEventSynchronize((hipEvent_t)ev)); }
int event_destroy(void* ev) { return check(hipEventDestroy((hipEvent_t)ev)); }
int stream_create(void** stream) {
    hipStream_t st = nullptr;
    if (check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking))) return -1;
    *stream = (void*)st;
    return 0;
}
int stream_destroy(void* stream) { return check(hipStreamDestroy((hipStream_t)stream)); }
// The address of `scratch` on the current device, looked up on the first call
// made with that device current and kept per device (each GPU has its own
// copy of the array at its own address).
int noalloc_scratch(void** out) {
    static std::mutex mu;
    static void* addr[IG_NOALLOC_MAX_DEVICES];
    int dev = -1;
    if (check(hipGetDevice(&dev))) return -1;
    if (dev < 0 || dev >= IG_NOALLOC_MAX_DEVICES) {
        snprintf(g_err, sizeof g_err, "device %d beyond the %d devices the scratch table covers", dev,
                 IG_NOALLOC_MAX_DEVICES);
        return -1;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)))) return -1;
        addr[dev] = p;
    }
    *out = addr[dev];
    return 0;
}
int launch_pack_instructions(const DevCtx* c, uint64_t first, uint64_t n, ig_instruction* out, void* stream) {
    if (!n) return 0;
    hipLaunchKernelGGL(ig_pack_instructions, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, c, first, n, out);
    return check(hipGetLastError());
}
int launch_pack_bindings(const DevCtx* c, uint64_t first, uint64_t n, ig_binding* out, void* stream) {
    if (!n) return 0;
    hipLaunchKernelGGL(ig_pack_bindings, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, c, first, n, out);
    return check(hipGetLastError());
}
int launch_pack_edges(const DevCtx* c, uint64_t first, uint64_t n, ig_edge* out, void* stream) {
    if (!n) return 0;
    hipLaunchKernelGGL(ig_pack_edges, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, c, first, n, out);
    return check(hipGetLastError());
}
int launch_stats(const DevCtx* c, uint64_t ni, uint64_t nb, uint64_t ne, DevStats* out, void* stream) {
    uint64_t m = ni > ne ? ni : ne;
    unsigned blocks = blocks_for(m > 0 ? m : 1, 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(ig_stats_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, c, ni, nb, ne, out);
    return check(hipGetLastError());
}
}  // namespace igrt
#endif  // IG_WIDE_ONLY
#endif  // IG_HOST_SIM
