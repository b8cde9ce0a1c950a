// ig_sim.cpp -- TEST BUILD ONLY: runs the kernels of ig_kernels.hip on the
// host, one workgroup emulated by std::threads and a barrier, so that the
// kernel logic can be checked (with host sanitizers) without a GPU.  The
// product library never contains this file.
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

#include "ig_kernels.hip"
#include "ig_ooo.hip"

unsigned long long ig_clock() {
    return (unsigned long long)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

namespace igsim {
thread_local ThreadCtx cur;
struct Barrier {
    std::mutex m;
    std::condition_variable cv;
    unsigned n = 0, count = 0, gen = 0;
    int line[1024];
    unsigned xchg[1024];
};
void barrier_wait(Barrier* b, int line) {
    b->line[cur.tid] = line;
    std::unique_lock<std::mutex> lk(b->m);
    const unsigned g = b->gen;
    if (++b->count == b->n) {
        b->count = 0;
        ++b->gen;
        b->cv.notify_all();
    } else if (!b->cv.wait_for(lk, std::chrono::seconds(20), [&] { return g != b->gen; })) {
        std::fprintf(stderr, "igsim: barrier timeout (thread %u of %u): threads diverged at a barrier\n", cur.tid,
                     cur.nthreads);
        for (unsigned t = 0; t < cur.nthreads; ++t) std::fprintf(stderr, "  thread %u last barrier at line %d\n", t, b->line[t]);
        std::abort();
    }
}
unsigned shfl_up(unsigned v, unsigned delta) {
    Barrier* b = cur.bar;
    b->xchg[cur.tid] = v;
    barrier_wait(b, -1);
    const unsigned lane = cur.tid % 64;
    const unsigned r = lane >= delta ? b->xchg[cur.tid - delta] : v;
    barrier_wait(b, -2);
    return r;
}
}  // namespace igsim

namespace igrt {
static char g_err[64] = "";
const char* last_error() { return g_err; }
int dev_malloc(void** p, size_t bytes) {
    *p = std::calloc(1, bytes + 256);
    return *p ? 0 : -1;
}
int dev_free(void* p) {
    std::free(p);
    return 0;
}
int host_malloc_pinned(void** p, size_t bytes) { return dev_malloc(p, bytes); }
int host_free_pinned(void* p) { return dev_free(p); }
int copy_h2d(void* dst, const void* src, size_t bytes, void*) {
    std::memcpy(dst, src, bytes);
    return 0;
}
int copy_d2h(void* dst, const void* src, size_t bytes, void*) {
    std::memcpy(dst, src, bytes);
    return 0;
}
int memset_d(void* dst, int v, size_t bytes, void*) {
    std::memset(dst, v, bytes);
    return 0;
}
int stream_sync(void*) { return 0; }
double clock_khz() { return 1e6; }

int launch_analyse(DevCtx* const* ptrs, unsigned n_blocks, unsigned threads, unsigned window, void*) {
    for (unsigned b = 0; b < n_blocks; ++b) {
        Shared* sh = new Shared();
        igsim::Barrier gate;
        gate.n = threads;
        for (int& l : gate.line) l = -1;
        std::vector<std::thread> ts;
        for (unsigned t = 0; t < threads; ++t)
            ts.emplace_back([=, &gate] {
                igsim::cur.tid = t;
                igsim::cur.nthreads = threads;
                igsim::cur.block = b;
                igsim::cur.bar = &gate;
                analyse(*ptrs[b], *sh, window);
            });
        for (auto& t : ts) t.join();
        delete sh;
    }
    return 0;
}

int launch_reset(DevCtx* const* ptrs, unsigned n, void*) {
    for (unsigned b = 0; b < n; ++b) reset_state(*ptrs[b], 0, 1);
    return 0;
}
int launch_gather(DevCtx* const* ptrs, unsigned n, uint64_t* out, void*) {
    for (unsigned i = 0; i < n; ++i) gather_progress(*ptrs[i], (u64*)out + 4 * (size_t)i);
    return 0;
}
// Launches of the emulation complete synchronously: events are always done.
int event_create(void** ev) {
    *ev = std::malloc(1);
    return *ev ? 0 : -1;
}
int event_record(void*, void*) { return 0; }
int event_query(void*) { return 1; }
int event_sync(void*) { return 0; }
int event_destroy(void* ev) {
    std::free(ev);
    return 0;
}
int stream_create(void** stream) {
    *stream = std::malloc(1);
    return *stream ? 0 : -1;
}
int stream_destroy(void* stream) {
    std::free(stream);
    return 0;
}
// The emulation's stand-in for the fixed device array of the no-alloc calls.
alignas(256) static unsigned char g_noalloc_scratch[IG_NOALLOC_SCRATCH_BYTES];
int noalloc_scratch(void** out) {
    *out = g_noalloc_scratch;
    return 0;
}
// A "graph" of the emulation: the recorded launch sequence, replayed.
struct SimGraph {
    std::vector<DevCtx*> ptrs;
    unsigned threads;
};
int graph_capture(DevCtx* const* ptrs, unsigned n, unsigned threads, void*, void** exec) {
    SimGraph* g = new SimGraph;
    g->ptrs.assign(ptrs, ptrs + n);
    g->threads = threads;
    *exec = g;
    return 0;
}
int graph_launch(void* exec, void* stream) {
    SimGraph* g = (SimGraph*)exec;
    launch_reset(g->ptrs.data(), (unsigned)g->ptrs.size(), stream);
    return launch_analyse(g->ptrs.data(), (unsigned)g->ptrs.size(), g->threads, 0, stream);
}
int graph_destroy(void* exec) {
    delete (SimGraph*)exec;
    return 0;
}

// The engine simulation: preparation as plain loops, then each graph's
// engine in one emulated workgroup.
int launch_ooo(const igd::OooGraph* gs, unsigned n_graphs, uint64_t, uint64_t, const ig_ooo_params* p, void*) {
    for (unsigned b = 0; b < n_graphs; ++b) {
        const igd::OooGraph& g = gs[b];
        igd::ooo_prep_tail(g);
        for (uint32_t x = 0; x < g.n; ++x) igd::ooo_prep_node(g, *p, x);
        for (uint32_t e = 0; e < g.ne; ++e) igd::ooo_prep_edge(g, e);
    }
    const unsigned threads = 16;  // the engine's logic does not depend on the workgroup size
    for (unsigned b = 0; b < n_graphs; ++b) {
        for (int phase = 0; phase < 2; ++phase) {
            igd::OooShared* sh = new igd::OooShared();
            std::vector<uint32_t> part(threads);
            igsim::Barrier gate;
            gate.n = threads;
            for (int& l : gate.line) l = -1;
            std::vector<std::thread> ts;
            for (unsigned t = 0; t < threads; ++t)
                ts.emplace_back([=, &gate, &part] {
                    igsim::cur.tid = t;
                    igsim::cur.nthreads = threads;
                    igsim::cur.block = b;
                    igsim::cur.bar = &gate;
                    if (phase == 0) igd::ooo_scan(gs[b], part.data());
                    else igd::ooo_engine(gs[b], *p, *sh);
                });
            for (auto& t : ts) t.join();
            delete sh;
            if (phase == 0)
                for (uint32_t e = 0; e < gs[b].ne; ++e) igd::ooo_fill_edge(gs[b], e);
        }
    }
    return 0;
}

int launch_pack_instructions(const DevCtx* c, uint64_t first, uint64_t n, ig_instruction* out, void*) {
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t x = first + i;
        ig_instruction r;
        std::memset(&r, 0, sizeof r);
        r.id = x;
        r.kind = c->i_kind[x];
        r.flags = c->i_flags[x];
        r.mem = c->i_mem[x];
        r.src_mem = c->i_src_mem[x];
        r.task = c->i_task[x];
        r.chunk = c->i_chunk[x];
        r.buffer = c->i_buffer[x];
        r.alloc = c->i_alloc[x];
        r.src_alloc = c->i_src_alloc[x];
        for (int d = 0; d < 3; ++d) {
            r.box.min[d] = c->i_box[d * c->cap_instr + x];
            r.box.max[d] = c->i_box[(3 + d) * c->cap_instr + x];
        }
        out[i] = r;
    }
    return 0;
}
int launch_pack_bindings(const DevCtx* c, uint64_t first, uint64_t n, ig_binding* out, void*) {
    for (uint64_t i = 0; i < n; ++i) {
        ig_binding r;
        std::memset(&r, 0, sizeof r);
        r.instr = c->b_instr[first + i];
        r.access = c->b_access[first + i];
        r.alloc = c->b_alloc[first + i];
        out[i] = r;
    }
    return 0;
}
int launch_pack_edges(const DevCtx* c, uint64_t first, uint64_t n, ig_edge* out, void*) {
    for (uint64_t i = 0; i < n; ++i) {
        ig_edge r;
        std::memset(&r, 0, sizeof r);
        r.from = c->e_from[first + i];
        r.to = c->e_to[first + i];
        r.kinds = c->e_kinds[first + i];
        out[i] = r;
    }
    return 0;
}
int launch_stats(const DevCtx* c, uint64_t ni, uint64_t nb, uint64_t ne, DevStats* out, void*) {
    for (uint64_t i = 0; i < ni; ++i) {
        u64 w[12];
        instr_words(*c, i, w);
        out->digest[0] += splitmix64(fnv_words(w, 12) ^ splitmix64(i));
        out->per_kind[c->i_kind[i] & 7] += 1;
    }
    for (uint64_t i = 0; i < nb; ++i) {
        u64 w[3] = {c->b_instr[i], c->b_access[i], c->b_alloc[i]};
        out->digest[1] += splitmix64(fnv_words(w, 3) ^ splitmix64(i));
    }
    for (uint64_t i = 0; i < ne; ++i) {
        u64 w[3] = {c->e_from[i], c->e_to[i], c->e_kinds[i]};
        out->digest[2] += splitmix64(fnv_words(w, 3) ^ splitmix64(i));
        for (int b = 0; b < 5; ++b)
            if (c->e_kinds[i] & (1u << b)) out->per_dep[b] += 1;
    }
    return 0;
}
}  // namespace igrt
