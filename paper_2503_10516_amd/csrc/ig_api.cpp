// ig_api.cpp -- host side of libig: argument validation, command recording,
// device-memory layout, launches and record fetch.  No analysis happens
// here; every step of instruction-graph generation runs in ig_kernels.hip.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ig_dev.h"

using namespace igd;

struct Caps {
    u32 nodes, devices, chunks, per_dev, n_dev, n_mem, mw;
    u32 horizon_step, lookahead, flush_horizons, queue_cap, threads, n_workers;
    u32 horizon_mode, horizon_max_tasks;
    u32 staging;
    u32 cap_cmds, cap_allocs, cap_queue, cap_heap, cap_rb, cap_unit, cap_scr, cap_src, cap_box;
    u64 cap_instr, cap_edges, cap_binds;
    u64 pack_bytes;
};

struct ig_context {
    ig_context_desc d;
    Caps k;
    DevCtx h;          // host view of the device context (device pointers)
    DevCtx* dctx;      // device copy
    DevCtx** dptrs;    // device array {dctx}
    DevStats* dstats;  // device
    void* pack;        // device staging for fetch
    char* arena;
    bool own_arena;
    u64 arena_bytes;
    void* stream;
    std::vector<DevCmd> cmds;
    size_t uploaded;
    struct HBuf {
        u32 dims;
        i64 ext[3];
        bool alive;
    };
    std::vector<HBuf> bufs;
    u64 n_tasks;
    bool shut;
    u64 cur_i, cur_b, cur_e, cur_t;
    Scalars s;
    bool s_valid;
    u64 launches;
};

static bool make_caps(const ig_context_desc* d, Caps& k) {
    if (!d || d->nodes == 0 || d->devices_per_node == 0) return false;
    if ((u64)d->nodes * d->devices_per_node > IG_MAX_DEVICES) return false;
    k.nodes = d->nodes;
    k.devices = d->devices_per_node;
    k.n_dev = k.nodes * k.devices;
    k.chunks = d->chunks ? d->chunks : k.n_dev;
    if (k.chunks % k.n_dev != 0 || k.chunks > MAX_CHUNKS) return false;
    k.per_dev = k.chunks / k.n_dev;
    k.n_mem = k.n_dev + 2;
    k.mw = (k.n_mem + 63) / 64;
    k.horizon_step = d->horizon_step ? d->horizon_step : 4;
    if (d->lookahead > 1) return false;
    k.lookahead = d->lookahead;
    k.flush_horizons = d->flush_horizons ? d->flush_horizons : 2;
    k.queue_cap = d->queue_cap;
    if (d->horizon_mode > 1) return false;
    k.horizon_mode = d->horizon_mode;
    k.horizon_max_tasks = d->horizon_max_tasks ? d->horizon_max_tasks : 16 * k.horizon_step;
    if (d->staging > 1) return false;
    k.staging = d->staging;
    k.threads = d->threads ? d->threads : 256;
    if (k.threads < 64 || k.threads > MAX_THREADS || (k.threads & 63)) return false;
    k.n_workers = std::min(k.threads, k.n_mem);
    k.cap_cmds = (u32)(d->cap_commands ? d->cap_commands : 65536);
    k.cap_instr = d->cap_instructions ? d->cap_instructions : (1ull << 20);
    k.cap_edges = d->cap_edges ? d->cap_edges : 4 * k.cap_instr;
    k.cap_binds = 2 * k.cap_instr + 64;
    if (k.cap_instr >= 0xFFFFFFF0ull || k.cap_edges >= (1ull << 40)) return false;
    k.cap_heap = (u32)(d->cap_state_words ? d->cap_state_words : (1u << 24));
    k.cap_rb = std::max<u32>(1024, k.cap_heap / 4);
    k.cap_unit = (u32)(d->cap_unit ? d->cap_unit : (1u << 18));
    k.cap_queue = 2 * k.cap_cmds + 2;
    k.cap_allocs = 1u << 16;
    k.cap_scr = (u32)(d->cap_scratch ? d->cap_scratch : 8192);
    if (d->cap_scratch && (d->cap_scratch < 256 || d->cap_scratch > (1u << 24))) return false;
    k.cap_src = k.cap_scr / 2;
    k.cap_box = k.cap_scr / 4;
    k.pack_bytes = 1ull << 24;
    return true;
}

struct Tail {
    DevCtx* dctx;
    DevCtx** dptrs;
    DevStats* dstats;
    void* pack;
};

// Lay out every device array of one context; with base == nullptr only the
// size is computed.
static u64 carve(const Caps& k, char* base, DevCtx* h, Tail* tail = nullptr) {
    u64 off = 0;
    auto take = [&](u64 bytes) -> char* {
        off = (off + 255) & ~255ull;
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
#define TAKE(field, type, count) h->field = (type*)take(sizeof(type) * (u64)(count))
    const u64 bm = (u64)MAX_BUF * k.n_mem;
    TAKE(cmds, DevCmd, k.cap_cmds);
    TAKE(i_kind, u8, k.cap_instr);
    TAKE(i_flags, u8, k.cap_instr);
    TAKE(i_mem, u16, k.cap_instr);
    TAKE(i_src_mem, u16, k.cap_instr);
    TAKE(i_task, u32, k.cap_instr);
    TAKE(i_chunk, u32, k.cap_instr);
    TAKE(i_buffer, u32, k.cap_instr);
    TAKE(i_alloc, u32, k.cap_instr);
    TAKE(i_src_alloc, u32, k.cap_instr);
    TAKE(i_box, i64, 6 * k.cap_instr);
    TAKE(e_from, u32, k.cap_edges);
    TAKE(e_to, u32, k.cap_edges);
    TAKE(e_kinds, u8, k.cap_edges);
    TAKE(b_instr, u32, k.cap_binds);
    TAKE(b_access, u32, k.cap_binds);
    TAKE(b_alloc, u32, k.cap_binds);
    TAKE(has_succ, u8, k.cap_instr);
    TAKE(task_status, i32, k.cap_cmds);
    TAKE(task_t0, u64, k.cap_cmds);
    TAKE(task_tq, u64, k.cap_cmds);
    TAKE(task_tc, u64, k.cap_cmds);
    TAKE(task_t1, u64, k.cap_cmds);
    TAKE(phase, u64, 32);
    TAKE(bufs, DBuf, MAX_BUF);
    TAKE(allocs, DAlloc, k.cap_allocs);
    TAKE(live_n, u32, bm);
    TAKE(live, u32, bm * MAX_LIVE);
    TAKE(plan_n, u32, bm);
    TAKE(plan, i64, bm * MAX_PLAN * 6);
    TAKE(queue, u32, k.cap_queue);
    TAKE(heap, u32, k.cap_heap);
    TAKE(heap_free, u32, 32);
    TAKE(rb, u32, (u64)k.cap_rb * 8);
    TAKE(rb_free, u64, k.n_mem);
    TAKE(reg, Region, (u64)MAX_CHUNKS * IG_MAX_ACCESS);
    TAKE(chunk_lo, i64, MAX_CHUNKS);
    TAKE(chunk_hi, i64, MAX_CHUNKS);
    TAKE(cons_off, u32, (u64)MAX_CHUNKS * IG_MAX_ACCESS);
    TAKE(cons_cnt, u32, (u64)MAX_CHUNKS * IG_MAX_ACCESS);
    TAKE(cons_x, u32, (u64)MAX_CHUNKS * IG_MAX_ACCESS);
    TAKE(k_rank, u32, (u64)MAX_CHUNKS);
    TAKE(big_n, u32, k.n_mem);
    TAKE(big_idx, u32, (u64)k.n_mem * MAX_BIG);
    TAKE(tm, u32, 4ull * k.n_mem);
    TAKE(copies, CopyRec, k.cap_unit);
    TAKE(dev_cnt, u32, k.n_dev);
    TAKE(dev_base, u32, k.n_dev);
    TAKE(kdev_cnt, u32, k.n_dev);
    TAKE(kdev_base, u32, k.n_dev);
    TAKE(inbox_cnt, u32, k.n_mem);
    TAKE(inbox_off, u32, k.n_mem);
    TAKE(inbox_cur, u32, k.n_mem);
    TAKE(inbox, InboxRec, k.cap_unit);
    TAKE(tab_off, u32, k.cap_unit + 1);
    TAKE(tab_cnt, u32, k.cap_unit + 1);
    TAKE(stage_from, u32, (u64)k.cap_unit * 8);
    TAKE(stage_kind, u8, (u64)k.cap_unit * 8);
    TAKE(pair_flag, u32, bm);
    TAKE(pair_cnt, u32, bm);
    TAKE(pair_acnt, u32, bm);
    TAKE(miss_n, u32, 4);
    TAKE(miss_val, i64, k.cap_scr);
    TAKE(miss_bd, u32, k.cap_scr);
    TAKE(remap, u32, 3ull * k.cap_scr);
    TAKE(wk_key, u64, (u64)k.n_workers * k.cap_scr);
    TAKE(wk_val, u32, (u64)k.n_workers * k.cap_scr);
    TAKE(wk_key2, u64, (u64)k.n_workers * k.cap_scr);
    TAKE(wk_val2, u32, (u64)k.n_workers * k.cap_scr);
    TAKE(wk_rsrc, u64, (u64)k.n_workers * RD_CACHE * k.cap_src);
    TAKE(wk_grp, RdGroup, (u64)k.n_workers * RD_CACHE);
    TAKE(wk_src, u64, (u64)k.threads * k.cap_src);  // any thread may stage a spilled source set
    TAKE(wk_src2, u64, (u64)k.threads * k.cap_src);
    TAKE(wk_box, i64, (u64)k.n_workers * k.cap_box * 6);
#undef TAKE
    Tail t;
    t.dctx = (DevCtx*)take(sizeof(DevCtx));         // the device copy of the context
    t.dptrs = (DevCtx**)take(sizeof(DevCtx*) * 2);  // pointer array for a single-context launch
    t.dstats = (DevStats*)take(sizeof(DevStats));
    t.pack = take(k.pack_bytes);                    // fetch staging
    if (tail) *tail = t;
    return (off + 255) & ~255ull;
}

static void fill_config(const Caps& k, DevCtx& h) {
    h.nodes = k.nodes;
    h.devices = k.devices;
    h.chunks = k.chunks;
    h.per_dev = k.per_dev;
    h.n_dev = k.n_dev;
    h.n_mem = k.n_mem;
    h.mw = k.mw;
    h.horizon_step = k.horizon_step;
    h.lookahead = k.lookahead;
    h.flush_horizons = k.flush_horizons;
    h.queue_cap = k.queue_cap;
    h.threads = k.threads;
    h.n_workers = k.n_workers;
    h.horizon_mode = k.horizon_mode;
    h.horizon_max_tasks = k.horizon_max_tasks;
    h.staging = k.staging;
    h.cap_cmds = k.cap_cmds;
    h.cap_allocs = k.cap_allocs;
    h.cap_queue = k.cap_queue;
    h.cap_heap = k.cap_heap;
    h.cap_rb = k.cap_rb;
    h.cap_unit = k.cap_unit;
    h.cap_scr = k.cap_scr;
    h.cap_src = k.cap_src;
    h.cap_box = k.cap_box;
    h.cap_instr = k.cap_instr;
    h.cap_edges = k.cap_edges;
    h.cap_binds = k.cap_binds;
    h.cmd_end = 0;
    std::memset(&h.s, 0, sizeof h.s);
}

template <class Rec, class Launch>
static ig_status fetch_records(ig_context* c, u64 total, u64& cursor, Rec* dst, size_t cap, size_t* n_out, Launch launch) {
    const u64 n = std::min<u64>(cap, total - cursor);
    const u64 per = c->k.pack_bytes / sizeof(Rec);
    u64 done = 0;
    while (done < n) {
        const u64 m = std::min(per, n - done);
        if (launch(cursor + done, m, (Rec*)c->pack) != 0) return IG_E_DEVICE;
        if (igrt::copy_d2h(dst + done, c->pack, m * sizeof(Rec), c->stream) != 0) return IG_E_DEVICE;
        if (igrt::stream_sync(c->stream) != 0) return IG_E_DEVICE;
        done += m;
    }
    cursor += n;
    if (n_out) *n_out = (size_t)n;
    return IG_OK;
}

extern "C" {

const char* ig_status_str(ig_status st) {
    switch (st) {
        case IG_OK: return "ok";
        case IG_W_UNINIT_READ: return "warning: read of uninitialised data";
        case IG_E_INVALID: return "invalid argument";
        case IG_E_OVERLAPPING_WRITE: return "overlapping writes";
        case IG_E_CAPACITY: return "capacity exceeded";
        case IG_E_DEVICE: return "device error";
        case IG_E_BUSY: return "busy";
        case IG_E_INTERNAL: return "internal invariant failed";
        default: return "unknown status";
    }
}

const char* ig_last_error(void) { return igrt::last_error(); }

ig_status ig_arena_bytes(const ig_context_desc* desc, uint64_t* bytes) {
    Caps k;
    if (!make_caps(desc, k) || !bytes) return IG_E_INVALID;
    DevCtx h;
    *bytes = carve(k, nullptr, &h);
    return IG_OK;
}

ig_status ig_context_create(const ig_context_desc* desc, ig_context** out) {
    Caps k;
    if (!out || !make_caps(desc, k)) return IG_E_INVALID;
    ig_context* c = new (std::nothrow) ig_context();
    if (!c) return IG_E_CAPACITY;
    c->d = *desc;
    c->k = k;
    c->stream = desc->stream;
    DevCtx probe;
    const u64 need = carve(k, nullptr, &probe);
    if (desc->arena) {
        if (desc->arena_bytes < need) {
            delete c;
            return IG_E_CAPACITY;
        }
        c->arena = (char*)desc->arena;
        c->own_arena = false;
    } else {
        void* p = nullptr;
        if (igrt::dev_malloc(&p, need) != 0) {
            delete c;
            return IG_E_DEVICE;
        }
        c->arena = (char*)p;
        c->own_arena = true;
    }
    c->arena_bytes = need;
    std::memset(&c->h, 0, sizeof c->h);
    Tail tail;
    carve(k, c->arena, &c->h, &tail);
    c->dctx = tail.dctx;
    c->dptrs = tail.dptrs;
    c->dstats = tail.dstats;
    c->pack = tail.pack;
    fill_config(k, c->h);
    if (igrt::memset_d(c->h.phase, 0, 32 * sizeof(u64), c->stream) != 0 ||
        igrt::copy_h2d(c->dctx, &c->h, sizeof(DevCtx), c->stream) != 0 ||
        igrt::copy_h2d(c->dptrs, &c->dctx, sizeof(DevCtx*), c->stream) != 0 ||
        igrt::stream_sync(c->stream) != 0) {
        if (c->own_arena) igrt::dev_free(c->arena);
        delete c;
        return IG_E_DEVICE;
    }
    c->uploaded = 0;
    c->n_tasks = 0;
    c->shut = false;
    c->cur_i = c->cur_b = c->cur_e = c->cur_t = 0;
    std::memset(&c->s, 0, sizeof c->s);
    c->s_valid = false;
    c->launches = 0;
    *out = c;
    return IG_OK;
}

ig_status ig_context_destroy(ig_context* c) {
    if (!c) return IG_E_INVALID;
    igrt::stream_sync(c->stream);
    if (c->own_arena) igrt::dev_free(c->arena);
    delete c;
    return IG_OK;
}

static bool can_record(ig_context* c) { return c && !c->shut && c->cmds.size() < c->k.cap_cmds; }

ig_status ig_buffer_create(ig_context* c, uint32_t dims, const int64_t extent[3], uint32_t elem_size, uint32_t init,
                           uint32_t* out_buffer) {
    if (!c || c->shut || !extent || dims < 1 || dims > 3 || elem_size == 0 || init > 1) return IG_E_INVALID;
    if (c->bufs.size() >= MAX_BUF || !can_record(c)) return IG_E_CAPACITY;
    DevCmd cmd;
    std::memset(&cmd, 0, sizeof cmd);
    cmd.kind = CMD_BUFFER;
    cmd.arg = (u32)c->bufs.size();
    cmd.dims = dims;
    cmd.elem_size = elem_size;
    cmd.init = init;
    ig_context::HBuf hb;
    hb.dims = dims;
    hb.alive = true;
    for (u32 d = 0; d < 3; ++d) {
        if (d < dims) {
            if (extent[d] < 1 || extent[d] > ((int64_t)1 << 40)) return IG_E_INVALID;
            cmd.ext[d] = extent[d];
        } else {
            cmd.ext[d] = 1;
        }
        hb.ext[d] = cmd.ext[d];
    }
    c->cmds.push_back(cmd);
    c->bufs.push_back(hb);
    if (out_buffer) *out_buffer = cmd.arg;
    return IG_OK;
}

ig_status ig_buffer_destroy(ig_context* c, uint32_t b) {
    if (!c || c->shut || b >= c->bufs.size() || !c->bufs[b].alive) return IG_E_INVALID;
    if (!can_record(c)) return IG_E_CAPACITY;
    DevCmd cmd;
    std::memset(&cmd, 0, sizeof cmd);
    cmd.kind = CMD_DESTROY;
    cmd.arg = b;
    c->cmds.push_back(cmd);
    c->bufs[b].alive = false;
    return IG_OK;
}

static ig_status validate_task(const ig_context* c, const ig_task_desc* t) {
    if (!t || t->dims < 1 || t->dims > 3 || t->n_access > IG_MAX_ACCESS) return IG_E_INVALID;
    const int64_t lim = (int64_t)1 << 40;
    for (u32 d = 0; d < 3; ++d) {
        if (d < t->dims) {
            if (t->box.min[d] > t->box.max[d] || t->box.min[d] < -lim || t->box.max[d] > lim) return IG_E_INVALID;
        } else if (t->box.min[d] != 0 || t->box.max[d] != 1) {
            return IG_E_INVALID;
        }
    }
    for (u32 j = 0; j < t->n_access; ++j) {
        const ig_access& a = t->access[j];
        if (a.buffer >= c->bufs.size() || !c->bufs[a.buffer].alive) return IG_E_INVALID;
        if (a.mode < 1 || a.mode > 3 || a.mapper > IG_MAP_FIXED) return IG_E_INVALID;
        const u32 bd = c->bufs[a.buffer].dims;
        const bool needs = a.mapper == IG_MAP_ONE_TO_ONE || a.mapper == IG_MAP_NEIGHBORHOOD || a.mapper == IG_MAP_SLICE;
        if (needs && bd != t->dims) return IG_E_INVALID;
        if (a.mapper == IG_MAP_SLICE && a.slice_dim >= bd) return IG_E_INVALID;
        if (a.mapper == IG_MAP_NEIGHBORHOOD)
            for (u32 d = 0; d < bd; ++d)
                if (a.radius[d] < 0 || a.radius[d] > lim) return IG_E_INVALID;
        if (a.mapper == IG_MAP_FIXED)
            for (u32 d = 0; d < bd; ++d)
                if (a.fixed.min[d] > a.fixed.max[d] || a.fixed.min[d] < -lim || a.fixed.max[d] > lim)
                    return IG_E_INVALID;
    }
    return IG_OK;
}

ig_status ig_submit_task(ig_context* c, const ig_task_desc* t, uint64_t* out_task) {
    if (!c || c->shut) return IG_E_INVALID;
    const ig_status v = validate_task(c, t);
    if (v != IG_OK) return v;
    if (!can_record(c)) return IG_E_CAPACITY;
    DevCmd cmd;
    std::memset(&cmd, 0, sizeof cmd);
    cmd.kind = CMD_TASK;
    cmd.arg = (u32)c->n_tasks;
    cmd.task = *t;
    // normalise the unused parts of the descriptor
    for (u32 j = t->n_access; j < IG_MAX_ACCESS; ++j) std::memset(&cmd.task.access[j], 0, sizeof(ig_access));
    c->cmds.push_back(cmd);
    if (out_task) *out_task = c->n_tasks;
    ++c->n_tasks;
    return IG_OK;
}

ig_status ig_submit_tasks(ig_context* c, const ig_task_desc* t, size_t n, uint64_t* out_first) {
    if (!c || (!t && n)) return IG_E_INVALID;
    if (out_first) *out_first = c->n_tasks;
    for (size_t i = 0; i < n; ++i) {
        const ig_status st = ig_submit_task(c, t + i, nullptr);
        if (st != IG_OK) return st;
    }
    return IG_OK;
}

static ig_status record_simple(ig_context* c, u32 kind) {
    if (!c || c->shut) return IG_E_INVALID;
    if (!can_record(c)) return IG_E_CAPACITY;
    DevCmd cmd;
    std::memset(&cmd, 0, sizeof cmd);
    cmd.kind = kind;
    c->cmds.push_back(cmd);
    return IG_OK;
}

ig_status ig_epoch(ig_context* c) { return record_simple(c, CMD_EPOCH); }

ig_status ig_shutdown(ig_context* c) {
    const ig_status st = record_simple(c, CMD_SHUTDOWN);
    if (st == IG_OK) {
        c->shut = true;
        for (auto& b : c->bufs) b.alive = false;
    }
    return st;
}

static ig_status upload(ig_context* c) {
    if (c->uploaded == c->cmds.size()) return IG_OK;
    // commands are appended only; a running analysis reads below cmd_end
    if (igrt::stream_sync(c->stream) != 0) return IG_E_DEVICE;
    const size_t n = c->cmds.size() - c->uploaded;
    if (igrt::copy_h2d(c->h.cmds + c->uploaded, c->cmds.data() + c->uploaded, n * sizeof(DevCmd), c->stream) != 0)
        return IG_E_DEVICE;
    const u32 end = (u32)c->cmds.size();
    if (igrt::copy_h2d(&c->dctx->cmd_end, &end, sizeof(u32), c->stream) != 0) return IG_E_DEVICE;
    if (igrt::stream_sync(c->stream) != 0) return IG_E_DEVICE;
    c->uploaded = c->cmds.size();
    c->h.cmd_end = end;
    return IG_OK;
}

ig_status ig_flush_window(ig_context* c) {
    if (!c) return IG_E_INVALID;
    const ig_status st = upload(c);
    if (st != IG_OK) return st;
    if (igrt::launch_analyse(c->dptrs, 1, c->k.threads, 0, c->stream) != 0) return IG_E_DEVICE;
    c->s_valid = false;
    ++c->launches;
    return IG_OK;
}

// The device table of context pointers for a batched launch, written into
// the first context's staging area (synchronously: the area is reused).
static ig_status put_table(ig_context* const* ctxs, size_t n, void* s, size_t extra_bytes, DevCtx*** out) {
    if (n * sizeof(DevCtx*) + extra_bytes > ctxs[0]->k.pack_bytes) return IG_E_CAPACITY;
    std::vector<DevCtx*> ptrs(n);
    for (size_t i = 0; i < n; ++i) ptrs[i] = ctxs[i]->dctx;
    DevCtx** table = (DevCtx**)ctxs[0]->pack;
    if (igrt::stream_sync(s) != 0) return IG_E_DEVICE;
    if (igrt::copy_h2d(table, ptrs.data(), n * sizeof(DevCtx*), s) != 0) return IG_E_DEVICE;
    if (igrt::stream_sync(s) != 0) return IG_E_DEVICE;
    *out = table;
    return IG_OK;
}

static ig_status check_batch(ig_context* const* ctxs, size_t n) {
    if (!ctxs || n == 0 || n > 0x7FFFFFFF) return IG_E_INVALID;
    for (size_t i = 0; i < n; ++i)
        if (!ctxs[i] || ctxs[i]->k.threads != ctxs[0]->k.threads) return IG_E_INVALID;
    return IG_OK;
}

static void mark_launched(ig_context* const* ctxs, size_t n, bool rewound) {
    for (size_t i = 0; i < n; ++i) {
        ig_context* c = ctxs[i];
        if (rewound) {
            c->cur_i = c->cur_b = c->cur_e = c->cur_t = 0;
            std::memset(&c->s, 0, sizeof c->s);
        }
        c->s_valid = false;
        ++c->launches;
    }
}

ig_status ig_batch_flush_window(ig_context* const* ctxs, size_t n, void* stream, uint32_t max_commands) {
    ig_status st = check_batch(ctxs, n);
    if (st != IG_OK) return st;
    for (size_t i = 0; i < n; ++i)
        if ((st = upload(ctxs[i])) != IG_OK) return st;
    void* s = stream ? stream : ctxs[0]->stream;
    DevCtx** table;
    if ((st = put_table(ctxs, n, s, 0, &table)) != IG_OK) return st;
    if (igrt::launch_analyse(table, (unsigned)n, ctxs[0]->k.threads, max_commands, s) != 0) return IG_E_DEVICE;
    mark_launched(ctxs, n, false);
    return IG_OK;
}

ig_status ig_batch_flush(ig_context* const* ctxs, size_t n, void* stream) {
    return ig_batch_flush_window(ctxs, n, stream, 0);
}

ig_status ig_batch_rewind(ig_context* const* ctxs, size_t n, void* stream) {
    ig_status st = check_batch(ctxs, n);
    if (st != IG_OK) return st;
    void* s = stream ? stream : ctxs[0]->stream;
    DevCtx** table;
    if ((st = put_table(ctxs, n, s, 0, &table)) != IG_OK) return st;
    if (igrt::launch_reset(table, (unsigned)n, s) != 0) return IG_E_DEVICE;
    for (size_t i = 0; i < n; ++i) {
        ig_context* c = ctxs[i];
        c->cur_i = c->cur_b = c->cur_e = c->cur_t = 0;
        std::memset(&c->s, 0, sizeof c->s);
        c->s_valid = false;
    }
    return IG_OK;
}

ig_status ig_batch_progress(ig_context* const* ctxs, size_t n, void* stream, ig_progress* out) {
    if (!out) return IG_E_INVALID;
    ig_status st = check_batch(ctxs, n);
    if (st != IG_OK) return st;
    void* s = stream ? stream : ctxs[0]->stream;
    const size_t tbytes = (n * sizeof(DevCtx*) + 255) & ~(size_t)255;
    DevCtx** table;
    if ((st = put_table(ctxs, n, s, tbytes + 32 * n, &table)) != IG_OK) return st;
    uint64_t* dev_out = (uint64_t*)((char*)ctxs[0]->pack + tbytes);
    std::vector<uint64_t> host(4 * n);
    if (igrt::launch_gather(table, (unsigned)n, dev_out, s) != 0) return IG_E_DEVICE;
    if (igrt::copy_d2h(host.data(), dev_out, 32 * n, s) != 0) return IG_E_DEVICE;
    if (igrt::stream_sync(s) != 0) return IG_E_DEVICE;
    for (size_t i = 0; i < n; ++i) {
        out[i].tasks_done = host[4 * i] & 0xFFFFFFFFu;
        out[i].tasks_seen = host[4 * i] >> 32;
        out[i].error = (int32_t)(uint32_t)(host[4 * i + 1] & 0xFFFFFFFFu);
        out[i].capacity_exceeded = (uint32_t)(host[4 * i + 1] >> 32);
        out[i].finished = (uint32_t)host[4 * i + 2];
        out[i].commands_done = (uint32_t)host[4 * i + 3];
    }
    return IG_OK;
}

static_assert(sizeof(ig_progress) == 32, "ig_progress doubles as 4 words of gather output");

ig_status ig_batch_progress_noalloc(ig_context* const* ctxs, size_t n, void* stream, ig_progress* out) {
    if (!out) return IG_E_INVALID;
    ig_status st = check_batch(ctxs, n);
    if (st != IG_OK) return st;
    if (n > IG_NOALLOC_MAX_CONTEXTS) return IG_E_CAPACITY;
    void* s = stream ? stream : ctxs[0]->stream;
    void* scr = nullptr;
    if (igrt::noalloc_scratch(&scr) != 0) return IG_E_DEVICE;
    DevCtx** table = (DevCtx**)scr;
    uint64_t* dev_out = (uint64_t*)((char*)scr + (size_t)IG_NOALLOC_MAX_CONTEXTS * sizeof(DevCtx*));
    // the caller's array stages the pointer table (8 of its 32 bytes per context)
    DevCtx** host_table = (DevCtx**)(void*)out;
    for (size_t i = 0; i < n; ++i) host_table[i] = ctxs[i]->dctx;
    if (igrt::copy_h2d(table, host_table, n * sizeof(DevCtx*), s) != 0) return IG_E_DEVICE;
    if (igrt::stream_sync(s) != 0) return IG_E_DEVICE;  // the staging is overwritten below
    if (igrt::launch_gather(table, (unsigned)n, dev_out, s) != 0) return IG_E_DEVICE;
    if (igrt::copy_d2h(out, dev_out, 32 * n, s) != 0) return IG_E_DEVICE;
    if (igrt::stream_sync(s) != 0) return IG_E_DEVICE;
    for (size_t i = 0; i < n; ++i) {
        u64 w[4];
        std::memcpy(w, (const char*)out + 32 * i, sizeof w);
        out[i].tasks_done = w[0] & 0xFFFFFFFFu;
        out[i].tasks_seen = w[0] >> 32;
        out[i].error = (int32_t)(uint32_t)(w[1] & 0xFFFFFFFFu);
        out[i].capacity_exceeded = (uint32_t)(w[1] >> 32);
        out[i].finished = (uint32_t)w[2];
        out[i].commands_done = (uint32_t)w[3];
    }
    return IG_OK;
}

struct ig_graph {
    std::vector<ig_context*> ctxs;
    void* table = nullptr;  // device copy of the context pointers (graph-owned)
    void* exec = nullptr;
};

ig_status ig_batch_graph_create(ig_context* const* ctxs, size_t n, void* stream, ig_graph** out) {
    if (!out) return IG_E_INVALID;
    ig_status st = check_batch(ctxs, n);
    if (st != IG_OK) return st;
    for (size_t i = 0; i < n; ++i)
        if ((st = upload(ctxs[i])) != IG_OK) return st;
    void* s = stream ? stream : ctxs[0]->stream;
    ig_graph* g = new ig_graph;
    g->ctxs.assign(ctxs, ctxs + n);
    std::vector<DevCtx*> ptrs(n);
    for (size_t i = 0; i < n; ++i) ptrs[i] = ctxs[i]->dctx;
    if (igrt::dev_malloc(&g->table, n * sizeof(DevCtx*)) != 0 ||
        igrt::copy_h2d(g->table, ptrs.data(), n * sizeof(DevCtx*), s) != 0 || igrt::stream_sync(s) != 0 ||
        igrt::graph_capture((DevCtx* const*)g->table, (unsigned)n, ctxs[0]->k.threads, s, &g->exec) != 0) {
        if (g->table) igrt::dev_free(g->table);
        delete g;
        return IG_E_DEVICE;
    }
    *out = g;
    return IG_OK;
}

ig_status ig_graph_launch(ig_graph* g, void* stream) {
    if (!g) return IG_E_INVALID;
    void* s = stream ? stream : g->ctxs[0]->stream;
    if (igrt::graph_launch(g->exec, s) != 0) return IG_E_DEVICE;
    mark_launched(g->ctxs.data(), g->ctxs.size(), true);
    return IG_OK;
}

ig_status ig_graph_destroy(ig_graph* g) {
    if (!g) return IG_E_INVALID;
    igrt::stream_sync(g->ctxs[0]->stream);
    const int rc = igrt::graph_destroy(g->exec);
    igrt::dev_free(g->table);
    delete g;
    return rc ? IG_E_DEVICE : IG_OK;
}

// ---------------------------------------------------------------------------
// Serving
// ---------------------------------------------------------------------------
struct ig_server {
    ig_server_desc d;
    void* side = nullptr;                  // stream for preparing admitted contexts
    std::vector<ig_context*> slot;         // nullptr: free
    std::vector<u64> bytes;                // arena bytes per slot
    std::vector<ig_session_progress> last; // latest collected progress per slot
    std::vector<int> inflight_n;           // queued launches covering the slot
    u64 used = 0;
    struct Launch {
        void* ev = nullptr;
        char* host = nullptr;              // pinned: table | progress words | cmd_end words | commands
        char* dev = nullptr;               // device: table | progress words
        std::vector<u32> slots;
        bool busy = false;
    };
    std::vector<Launch> ring;
    size_t next = 0;                       // ring entry of the next launch
    size_t oldest = 0;                     // ring entry of the oldest queued launch
    size_t queued = 0;
    u64 host_bytes = 0, dev_bytes = 0;
};

static size_t srv_table_bytes(const ig_server* s) { return ((size_t)s->d.slots * sizeof(DevCtx*) + 255) & ~(size_t)255; }
static size_t srv_prog_bytes(const ig_server* s) { return ((size_t)s->d.slots * 32 + 255) & ~(size_t)255; }
static size_t srv_end_bytes(const ig_server* s) { return ((size_t)s->d.slots * 4 + 255) & ~(size_t)255; }

static void srv_free(ig_server* s) {
    for (auto& L : s->ring) {
        if (L.ev) igrt::event_destroy(L.ev);
        if (L.host) igrt::host_free_pinned(L.host);
        if (L.dev) igrt::dev_free(L.dev);
    }
    if (s->side) igrt::stream_destroy(s->side);
    delete s;
}

ig_status ig_server_create(const ig_server_desc* desc, ig_server** out) {
    if (!desc || !out || desc->slots == 0 || desc->slots > 4096 || desc->max_inflight > 8) return IG_E_INVALID;
    const u32 threads = desc->threads ? desc->threads : 256;
    if (threads < 64 || threads > MAX_THREADS || (threads & 63)) return IG_E_INVALID;
    ig_server* s = new (std::nothrow) ig_server();
    if (!s) return IG_E_CAPACITY;
    s->d = *desc;
    s->d.threads = threads;
    s->d.max_inflight = desc->max_inflight ? desc->max_inflight : 2;
    s->d.stage_bytes = std::max<u64>(desc->stage_bytes ? desc->stage_bytes : (8ull << 20), sizeof(DevCmd));
    s->slot.assign(s->d.slots, nullptr);
    s->bytes.assign(s->d.slots, 0);
    s->last.assign(s->d.slots, ig_session_progress{});
    s->inflight_n.assign(s->d.slots, 0);
    s->host_bytes = srv_table_bytes(s) + srv_prog_bytes(s) + srv_end_bytes(s) + s->d.stage_bytes;
    s->dev_bytes = srv_table_bytes(s) + srv_prog_bytes(s);
    s->ring.resize(s->d.max_inflight);
    if (igrt::stream_create(&s->side) != 0) {
        s->side = nullptr;
        srv_free(s);
        return IG_E_DEVICE;
    }
    for (auto& L : s->ring) {
        void* h = nullptr;
        void* dv = nullptr;
        if (igrt::event_create(&L.ev) != 0) L.ev = nullptr;
        if (igrt::host_malloc_pinned(&h, s->host_bytes) == 0) L.host = (char*)h;
        if (igrt::dev_malloc(&dv, s->dev_bytes) == 0) L.dev = (char*)dv;
        if (!L.ev || !L.host || !L.dev) {
            srv_free(s);
            return IG_E_DEVICE;
        }
    }
    *out = s;
    return IG_OK;
}

ig_status ig_server_destroy(ig_server* s) {
    if (!s) return IG_E_INVALID;
    for (auto& L : s->ring)
        if (L.busy) igrt::event_sync(L.ev);
    igrt::stream_sync(s->d.stream);
    for (ig_context* c : s->slot)
        if (c) ig_context_destroy(c);
    srv_free(s);
    return IG_OK;
}

ig_status ig_server_admit(ig_server* s, const ig_context_desc* desc, uint32_t* out_slot) {
    if (!s || !desc || !out_slot) return IG_E_INVALID;
    if (desc->threads && desc->threads != s->d.threads) return IG_E_INVALID;
    ig_context_desc d = *desc;
    d.threads = s->d.threads;
    d.stream = s->side;
    uint64_t need = 0;
    const ig_status st = ig_arena_bytes(&d, &need);
    if (st != IG_OK) return st;
    u32 free_slot = NONE;
    for (u32 i = 0; i < s->d.slots && free_slot == NONE; ++i)
        if (!s->slot[i]) free_slot = i;
    if (free_slot == NONE) return IG_E_BUSY;
    if (s->d.arena_budget && s->used + need > s->d.arena_budget) return IG_E_BUSY;
    ig_context* c = nullptr;
    const ig_status cs = ig_context_create(&d, &c);  // prepared (and synchronised) on the side stream
    if (cs != IG_OK) return cs;
    c->stream = s->d.stream;
    s->slot[free_slot] = c;
    s->bytes[free_slot] = need;
    s->used += need;
    s->inflight_n[free_slot] = 0;
    ig_session_progress& p = s->last[free_slot];
    std::memset(&p, 0, sizeof p);
    p.slot = free_slot;
    *out_slot = free_slot;
    return IG_OK;
}

ig_status ig_server_session(ig_server* s, uint32_t slot, ig_context** out) {
    if (!s || !out || slot >= s->d.slots || !s->slot[slot]) return IG_E_INVALID;
    *out = s->slot[slot];
    return IG_OK;
}

ig_status ig_server_submit(ig_server* s, uint32_t slot, const ig_task_desc* task, uint64_t* out_task) {
    if (!s || slot >= s->d.slots || !s->slot[slot]) return IG_E_INVALID;
    return ig_submit_task(s->slot[slot], task, out_task);
}

ig_status ig_server_detach(ig_server* s, uint32_t slot, ig_context** out) {
    if (!s || !out || slot >= s->d.slots || !s->slot[slot]) return IG_E_INVALID;
    if (s->inflight_n[slot]) return IG_E_BUSY;
    ig_context* c = s->slot[slot];
    // a detached context is used on its own from now on: progress known,
    // scalars read afresh
    c->s_valid = false;
    s->slot[slot] = nullptr;
    s->used -= s->bytes[slot];
    s->bytes[slot] = 0;
    *out = c;
    return IG_OK;
}

// Collect the oldest queued launch (its event has completed).
static void srv_collect(ig_server* s) {
    ig_server::Launch& L = s->ring[s->oldest];
    const u64* w = (const u64*)(L.host + srv_table_bytes(s));
    for (size_t i = 0; i < L.slots.size(); ++i) {
        const u32 q = L.slots[i];
        s->inflight_n[q] -= 1;
        if (!s->slot[q]) continue;
        ig_session_progress& p = s->last[q];
        p.tasks_done = w[4 * i] & 0xFFFFFFFFu;
        p.tasks_seen = w[4 * i] >> 32;
        p.error = (int32_t)(uint32_t)(w[4 * i + 1] & 0xFFFFFFFFu);
        p.finished = (uint32_t)w[4 * i + 2];
        p.commands_done = (uint32_t)w[4 * i + 3];
    }
    L.busy = false;
    L.slots.clear();
    s->oldest = (s->oldest + 1) % s->ring.size();
    s->queued -= 1;
}

// Queue one launch over the sessions with commands no queued launch covers.
static ig_status srv_launch(ig_server* s, bool* launched) {
    *launched = false;
    ig_server::Launch& L = s->ring[s->next];
    char* table_h = L.host;
    char* end_h = L.host + srv_table_bytes(s) + srv_prog_bytes(s);
    char* stage = end_h + srv_end_bytes(s);
    u64 stage_used = 0;
    std::vector<DevCtx*> ptrs;
    L.slots.clear();
    for (u32 q = 0; q < s->d.slots; ++q) {
        ig_context* c = s->slot[q];
        if (!c) continue;
        // new commands go into this launch (launches of one stream run in
        // order); commands a collected launch left unanalysed (the window)
        // go in only while no queued launch covers the session
        const size_t rec = c->cmds.size();
        const bool unanalysed = !s->inflight_n[q] && s->last[q].commands_done < c->uploaded;
        size_t n = rec - c->uploaded;
        if (n == 0 && !unanalysed) continue;
        const u64 room = (s->d.stage_bytes - stage_used) / sizeof(DevCmd);
        if (n > room) n = (size_t)room;
        if (n == 0 && !unanalysed) continue;
        if (n) {
            std::memcpy(stage + stage_used, c->cmds.data() + c->uploaded, n * sizeof(DevCmd));
            if (igrt::copy_h2d(c->h.cmds + c->uploaded, stage + stage_used, n * sizeof(DevCmd), s->d.stream) != 0)
                return IG_E_DEVICE;
            stage_used += n * sizeof(DevCmd);
            c->uploaded += n;
            u32* endw = (u32*)end_h + L.slots.size();
            *endw = (u32)c->uploaded;
            if (igrt::copy_h2d(&c->dctx->cmd_end, endw, sizeof(u32), s->d.stream) != 0) return IG_E_DEVICE;
            c->h.cmd_end = (u32)c->uploaded;
        }
        ptrs.push_back(c->dctx);
        L.slots.push_back(q);
    }
    if (L.slots.empty()) return IG_OK;
    std::memcpy(table_h, ptrs.data(), ptrs.size() * sizeof(DevCtx*));
    DevCtx** table_d = (DevCtx**)L.dev;
    uint64_t* prog_d = (uint64_t*)(L.dev + srv_table_bytes(s));
    char* prog_h = L.host + srv_table_bytes(s);
    const unsigned n = (unsigned)L.slots.size();
    if (igrt::copy_h2d(table_d, table_h, n * sizeof(DevCtx*), s->d.stream) != 0 ||
        igrt::launch_analyse(table_d, n, s->d.threads, s->d.window, s->d.stream) != 0 ||
        igrt::launch_gather(table_d, n, prog_d, s->d.stream) != 0 ||
        igrt::copy_d2h(prog_h, prog_d, 32ull * n, s->d.stream) != 0 || igrt::event_record(L.ev, s->d.stream) != 0)
        return IG_E_DEVICE;
    for (u32 q : L.slots) {
        s->inflight_n[q] += 1;
        s->slot[q]->s_valid = false;
        s->slot[q]->launches += 1;
    }
    L.busy = true;
    s->next = (s->next + 1) % s->ring.size();
    s->queued += 1;
    *launched = true;
    return IG_OK;
}

ig_status ig_server_poll(ig_server* s, uint32_t wait, ig_session_progress* out, size_t cap, size_t* n_out) {
    if (!s || (!out && cap)) return IG_E_INVALID;
    if (wait && s->queued && igrt::event_sync(s->ring[s->oldest].ev) != 0) return IG_E_DEVICE;
    while (s->queued) {
        const int q = igrt::event_query(s->ring[s->oldest].ev);
        if (q < 0) return IG_E_DEVICE;
        if (q == 0) break;
        srv_collect(s);
    }
    while (s->queued < s->ring.size()) {
        bool launched = false;
        const ig_status st = srv_launch(s, &launched);
        if (st != IG_OK) return st;
        if (!launched) break;
    }
    size_t k = 0;
    for (u32 q = 0; q < s->d.slots && k < cap; ++q) {
        if (!s->slot[q]) continue;
        ig_session_progress p = s->last[q];
        p.slot = q;
        p.in_flight = s->inflight_n[q] ? 1 : 0;
        p.commands_recorded = (uint32_t)s->slot[q]->cmds.size();
        out[k++] = p;
    }
    if (n_out) *n_out = k;
    return IG_OK;
}

static ig_status refresh(ig_context* c) {
    if (c->s_valid) return IG_OK;
    if (igrt::stream_sync(c->stream) != 0) return IG_E_DEVICE;
    if (igrt::copy_d2h(&c->s, &c->dctx->s, sizeof(Scalars), c->stream) != 0) return IG_E_DEVICE;
    if (igrt::stream_sync(c->stream) != 0) return IG_E_DEVICE;
    c->s_valid = true;
    return IG_OK;
}

ig_status ig_sync(ig_context* c) {
    if (!c) return IG_E_INVALID;
    const ig_status st = refresh(c);
    if (st != IG_OK) return st;
    if (c->s.error) return c->s.error;
    return IG_OK;
}

ig_status ig_rewind(ig_context* c) {
    if (!c) return IG_E_INVALID;
    if (igrt::launch_reset(c->dptrs, 1, c->stream) != 0) return IG_E_DEVICE;
    c->cur_i = c->cur_b = c->cur_e = c->cur_t = 0;
    std::memset(&c->s, 0, sizeof c->s);
    c->s_valid = false;
    return IG_OK;
}

ig_status ig_counts(ig_context* c, uint64_t* ni, uint64_t* nb, uint64_t* ne, uint64_t* nt) {
    if (!c) return IG_E_INVALID;
    const ig_status st = refresh(c);
    if (st != IG_OK) return st;
    if (ni) *ni = c->s.n_instr;
    if (nb) *nb = c->s.n_binds;
    if (ne) *ne = c->s.n_edges;
    if (nt) *nt = c->s.n_tasks;
    return IG_OK;
}

ig_status ig_fetch_instructions(ig_context* c, ig_instruction* dst, size_t cap, size_t* n_out) {
    if (!c || (!dst && cap)) return IG_E_INVALID;
    const ig_status st = refresh(c);
    if (st != IG_OK) return st;
    return fetch_records(c, c->s.n_instr, c->cur_i, dst, cap, n_out, [&](u64 first, u64 m, ig_instruction* out) {
        return igrt::launch_pack_instructions(c->dctx, first, m, out, c->stream);
    });
}

ig_status ig_fetch_bindings(ig_context* c, ig_binding* dst, size_t cap, size_t* n_out) {
    if (!c || (!dst && cap)) return IG_E_INVALID;
    const ig_status st = refresh(c);
    if (st != IG_OK) return st;
    return fetch_records(c, c->s.n_binds, c->cur_b, dst, cap, n_out, [&](u64 first, u64 m, ig_binding* out) {
        return igrt::launch_pack_bindings(c->dctx, first, m, out, c->stream);
    });
}

ig_status ig_fetch_edges(ig_context* c, ig_edge* dst, size_t cap, size_t* n_out) {
    if (!c || (!dst && cap)) return IG_E_INVALID;
    const ig_status st = refresh(c);
    if (st != IG_OK) return st;
    return fetch_records(c, c->s.n_edges, c->cur_e, dst, cap, n_out, [&](u64 first, u64 m, ig_edge* out) {
        return igrt::launch_pack_edges(c->dctx, first, m, out, c->stream);
    });
}

ig_status ig_fetch_task_status(ig_context* c, int32_t* dst, size_t cap, size_t* n_out) {
    if (!c || (!dst && cap)) return IG_E_INVALID;
    const ig_status st = refresh(c);
    if (st != IG_OK) return st;
    const u64 n = std::min<u64>(cap, c->s.n_tasks - c->cur_t);
    if (n) {
        if (igrt::copy_d2h(dst, c->h.task_status + c->cur_t, n * sizeof(int32_t), c->stream) != 0) return IG_E_DEVICE;
        if (igrt::stream_sync(c->stream) != 0) return IG_E_DEVICE;
    }
    c->cur_t += n;
    if (n_out) *n_out = (size_t)n;
    return IG_OK;
}

ig_status ig_fetch_task_times(ig_context* c, double* dst, size_t cap, size_t* n_out) {
    if (!c || (!dst && cap)) return IG_E_INVALID;
    const ig_status st = refresh(c);
    if (st != IG_OK) return st;
    const u64 n = std::min<u64>(cap, c->s.n_tasks);
    std::vector<u64> t[4];
    u64* src[4] = {c->h.task_t0, c->h.task_tq, c->h.task_tc, c->h.task_t1};
    for (int q = 0; q < 4; ++q) {
        t[q].resize(n);
        if (n && igrt::copy_d2h(t[q].data(), src[q], n * sizeof(u64), c->stream) != 0) return IG_E_DEVICE;
    }
    if (n && igrt::stream_sync(c->stream) != 0) return IG_E_DEVICE;
    const double khz = igrt::clock_khz();
    if (khz <= 0) return IG_E_DEVICE;
    for (u64 i = 0; i < n; ++i)
        for (int q = 0; q < 4; ++q) dst[4 * i + q] = (double)(t[q][i] - t[0][0]) / khz * 1e6;
    if (n_out) *n_out = (size_t)n;
    return IG_OK;
}

ig_status ig_stats_get(ig_context* c, ig_stats* out) {
    if (!c || !out) return IG_E_INVALID;
    ig_status st = refresh(c);
    if (st != IG_OK) return st;
    if (igrt::memset_d(c->dstats, 0, sizeof(DevStats), c->stream) != 0) return IG_E_DEVICE;
    if (igrt::launch_stats(c->dctx, c->s.n_instr, c->s.n_binds, c->s.n_edges, c->dstats, c->stream) != 0)
        return IG_E_DEVICE;
    DevStats ds;
    if (igrt::copy_d2h(&ds, c->dstats, sizeof ds, c->stream) != 0) return IG_E_DEVICE;
    if (igrt::stream_sync(c->stream) != 0) return IG_E_DEVICE;
    std::memset(out, 0, sizeof *out);
    out->n_instructions = c->s.n_instr;
    out->n_bindings = c->s.n_binds;
    out->n_edges = c->s.n_edges;
    for (int i = 0; i < 8; ++i) out->per_kind[i] = ds.per_kind[i];
    for (int i = 0; i < 5; ++i) out->per_dep[i] = ds.per_dep[i];
    out->resizes = c->s.resizes;
    out->warnings = c->s.warnings;
    out->tasks_submitted = c->n_tasks;
    out->tasks_rejected = c->s.rejected;
    out->digest_instructions = ds.digest[0];
    out->digest_bindings = ds.digest[1];
    out->digest_edges = ds.digest[2];
    out->commands_analysed = c->s.cmd_next;
    out->launches = c->launches;
    out->state_words_used = c->s.heap_top;
    out->reader_blocks_used = c->s.rb_top;
    out->capacity_exceeded = c->s.error == IG_E_CAPACITY ? c->s.cap_what : 0;
    u64 ph[32];
    if (igrt::copy_d2h(ph, c->h.phase, sizeof ph, c->stream) != 0 || igrt::stream_sync(c->stream) != 0)
        return IG_E_DEVICE;
    const double khz = igrt::clock_khz();
    for (int i = 0; i < 16; ++i) {
        out->phase_us[i] = khz > 0 ? (double)ph[i] / khz * 1e3 : 0.0;
        out->phase_count[i] = ph[16 + i];
    }
    return IG_OK;
}

// ---------------------------------------------------------------------------
// Out-of-order engine simulation (Sec. 4.1) over the contexts' graphs.
// ---------------------------------------------------------------------------
struct ig_ooo {
    ig_ooo_params p;
    std::vector<OooGraph> g;  // host view (device pointers)
    OooGraph* dg;             // device array
    ig_ooo_summary* dsum;
    i32* dstatus;
    char* mem;                // one device allocation for all of the above
    u64 max_n, max_ne;
    void* stream;             // of the last run
    bool ran;
};

static bool ooo_params_ok(const ig_ooo_params* p) {
    if (!p || p->lanes_per_device == 0 || p->host_lanes == 0 || p->window == 0 || p->window > IG_OOO_MAX_WINDOW ||
        p->eager > 1)
        return false;
    if ((u64)p->devices * p->lanes_per_device + p->host_lanes > IG_OOO_MAX_LANES) return false;
    return p->kernel_ns && p->copy_ns && p->alloc_ns && p->free_ns;
}

static u64 al256(u64 b) { return (b + 255) & ~(u64)255; }

ig_status ig_ooo_create(ig_context* const* ctxs, size_t n, const ig_ooo_params* p, ig_ooo** out) {
    if (!out) return IG_E_INVALID;
    *out = nullptr;
    if (!ctxs || n == 0 || n > 65535 || !ooo_params_ok(p)) return IG_E_INVALID;
    u64 bytes = al256(n * sizeof(OooGraph)) + al256(n * sizeof(ig_ooo_summary)) + al256(n * sizeof(i32));
    for (size_t i = 0; i < n; ++i) {
        if (!ctxs[i]) return IG_E_INVALID;
        const ig_status st = refresh(ctxs[i]);
        if (st != IG_OK) return st;
        const Scalars& sc = ctxs[i]->s;
        if (sc.error || sc.n_instr > 0x7FFFFFFFull || sc.n_edges > 0xFFFFFFFFull) return IG_E_INVALID;
        const u64 m = sc.n_instr, e = sc.n_edges;
        bytes += al256(m * sizeof(ig_ooo_slot)) + al256((m + 1) * 4) + al256(e * 4) + al256(m * sizeof(OooRec)) +
                 al256(m * sizeof(OooCnt)) + al256(m * 4) + al256(m * 8);
    }
    ig_ooo* o = new ig_ooo();
    o->p = *p;
    if (igrt::dev_malloc((void**)&o->mem, bytes) != 0) {
        delete o;
        return IG_E_DEVICE;
    }
    char* cur = o->mem;
    auto take = [&](u64 b) {
        char* r = cur;
        cur += al256(b);
        return r;
    };
    o->dg = (OooGraph*)take(n * sizeof(OooGraph));
    o->dsum = (ig_ooo_summary*)take(n * sizeof(ig_ooo_summary));
    o->dstatus = (i32*)take(n * sizeof(i32));
    o->g.resize(n);
    for (size_t i = 0; i < n; ++i) {
        const ig_context* c = ctxs[i];
        OooGraph& g = o->g[i];
        std::memset(&g, 0, sizeof g);
        g.kind = c->h.i_kind;
        g.flags = c->h.i_flags;
        g.mem = c->h.i_mem;
        g.box = c->h.i_box;
        g.e_from = c->h.e_from;
        g.e_to = c->h.e_to;
        g.box_stride = c->h.cap_instr;
        g.n = (u32)c->s.n_instr;
        g.ne = (u32)c->s.n_edges;
        g.sum = o->dsum + i;
        g.status = o->dstatus + i;
        g.out = (ig_ooo_slot*)take((u64)g.n * sizeof(ig_ooo_slot));
        g.out_off = (u32*)take(((u64)g.n + 1) * 4);
        g.out_adj = (u32*)take((u64)g.ne * 4);
        g.cnt = (OooCnt*)take((u64)g.n * sizeof(OooCnt));
        g.rec = (OooRec*)take((u64)g.n * sizeof(OooRec));
        g.cls = (u32*)take((u64)g.n * 4);
        g.dur = (u64*)take((u64)g.n * 8);
        o->max_n = std::max<u64>(o->max_n, g.n);
        o->max_ne = std::max<u64>(o->max_ne, g.ne);
    }
    if (igrt::copy_h2d(o->dg, o->g.data(), n * sizeof(OooGraph), nullptr) != 0 || igrt::stream_sync(nullptr) != 0) {
        igrt::dev_free(o->mem);
        delete o;
        return IG_E_DEVICE;
    }
    *out = o;
    return IG_OK;
}

ig_status ig_ooo_run(ig_ooo* o, void* stream) {
    if (!o) return IG_E_INVALID;
    if (igrt::memset_d(o->dstatus, 0, o->g.size() * sizeof(i32), stream) != 0) return IG_E_DEVICE;
    if (igrt::launch_ooo(o->dg, (unsigned)o->g.size(), o->max_n, o->max_ne, &o->p, stream) != 0) return IG_E_DEVICE;
    o->stream = stream;
    o->ran = true;
    return IG_OK;
}

ig_status ig_ooo_slots(ig_ooo* o, size_t i, ig_ooo_slot** d_slots, uint64_t* n) {
    if (!o || i >= o->g.size() || !d_slots) return IG_E_INVALID;
    *d_slots = o->g[i].out;
    if (n) *n = o->g[i].n;
    return IG_OK;
}

ig_status ig_ooo_fetch(ig_ooo* o, size_t i, ig_ooo_slot* dst, size_t cap, size_t* n_out, ig_ooo_summary* sum) {
    if (!o || i >= o->g.size() || (!dst && cap) || !o->ran) return IG_E_INVALID;
    const OooGraph& g = o->g[i];
    i32 st = 0;
    ig_ooo_summary hs;
    const size_t m = std::min<size_t>(cap, g.n);
    if (igrt::stream_sync(o->stream) != 0 || igrt::copy_d2h(&st, g.status, sizeof st, o->stream) != 0 ||
        igrt::copy_d2h(&hs, g.sum, sizeof hs, o->stream) != 0 ||
        (m && igrt::copy_d2h(dst, g.out, m * sizeof(ig_ooo_slot), o->stream) != 0) || igrt::stream_sync(o->stream) != 0)
        return IG_E_DEVICE;
    if (sum) *sum = hs;
    if (n_out) *n_out = m;
    return st;
}

ig_status ig_ooo_destroy(ig_ooo* o) {
    if (!o) return IG_E_INVALID;
    if (o->ran) igrt::stream_sync(o->stream);
    igrt::dev_free(o->mem);
    delete o;
    return IG_OK;
}

}  // extern "C"
