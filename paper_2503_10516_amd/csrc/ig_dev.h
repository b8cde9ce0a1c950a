// ig_dev.h -- device-side data layout of libig (instruction-graph generation).
//
// One stream (context) is analysed by ONE workgroup.  Its state lives in
// device memory, described by DevCtx:
//   * the recorded command log (buffer creation, tasks, epochs, destroys);
//   * output records as structure-of-arrays (instructions, bindings, edges)
//     plus one "has successor" byte per instruction (execution front);
//   * per buffer a coordinate-compressed cell grid: the sorted coordinates at
//     which any accessed region, allocation or buffer boundary starts or ends,
//     per dimension.  Every region the analysis ever handles is a union of
//     grid cells, so region maps are dense arrays over cells:
//       buffer map   (per cell)  original producer, producer memory,
//                                up-to-date memory mask        (Sec. 3.3)
//       init map     (per cell)  initialised?                  (Sec. 4.4)
//       allocation map (per cell of the allocation) last writer and the
//                                head of a reader list          (Sec. 3.2)
//     Grids are refined (cells split) when a task brings a new coordinate.
//   * horizon/epoch substitution (Sec. 3.5) is applied lazily: an id below
//     the current synchronisation point S reads as S, a reader below the last
//     epoch E reads as absent; this equals rewriting every map eagerly.
//
// Work inside the workgroup is split by *memory*: the worker thread owning a
// simulated memory performs every update of that memory's allocations, so
// allocation maps need no atomics.  The one cross-memory effect (a coherence
// copy reading a source allocation on another memory) is routed through a
// per-memory inbox and applied by the owner after the copy phase.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "ig.h"

#ifdef IG_HOST_SIM
// ---------------------------------------------------------------------------
// Host emulation of one workgroup (test build only: std::threads + barrier).
// The product library is always the HIP build; this exists so that the kernel
// logic can be exercised and bounds-checked on a machine without a GPU.
// ---------------------------------------------------------------------------
#include <atomic>
#include <cstring>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
namespace igsim {
struct Barrier;
struct ThreadCtx {
    unsigned tid, nthreads, block;
    Barrier* bar;
};
extern thread_local ThreadCtx cur;
void barrier_wait(Barrier* b, int line);
unsigned shfl_up(unsigned v, unsigned delta);  // 64-lane wave shuffle, emulated
}  // namespace igsim
inline unsigned ig_tid() { return igsim::cur.tid; }
inline unsigned ig_nthreads() { return igsim::cur.nthreads; }
inline unsigned ig_block() { return igsim::cur.block; }
inline void ig_barrier_at(int line) { igsim::barrier_wait(igsim::cur.bar, line); }
inline unsigned ig_shfl_up(unsigned v, unsigned delta) { return igsim::shfl_up(v, delta); }
inline unsigned atomicAdd(unsigned* p, unsigned v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline unsigned long long atomicOr(unsigned long long* p, unsigned long long v) {
    return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST);
}
inline unsigned atomicOr(unsigned* p, unsigned v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicExch(unsigned* p, unsigned v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicMax(unsigned* p, unsigned v) {
    unsigned cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (cur < v && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return cur;
}
inline unsigned long long atomicMax(unsigned long long* p, unsigned long long v) {
    unsigned long long cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (cur < v && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return cur;
}
inline unsigned long long atomicMin(unsigned long long* p, unsigned long long v) {
    unsigned long long cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (cur > v && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return cur;
}
inline unsigned atomicCAS(unsigned* p, unsigned cmp, unsigned v) {
    __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
    return cmp;
}
inline unsigned long long atomicCAS(unsigned long long* p, unsigned long long cmp, unsigned long long v) {
    __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
    return cmp;
}
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __threadfence_block() { std::atomic_thread_fence(std::memory_order_seq_cst); }
unsigned long long ig_clock();
#define IGD inline
#define IGN
// bounds checks of per-thread scratch, active in the host emulation only
#include <cstdio>
#include <cstdlib>
#define IG_SIM_CHECK(cond, what)                                                   \
    do {                                                                           \
        if (!(cond)) {                                                             \
            std::fprintf(stderr, "ig sim: %s violated at line %d\n", what, __LINE__); \
            std::abort();                                                          \
        }                                                                          \
    } while (0)
#else
#define IG_SIM_CHECK(cond, what) ((void)0)
#include <hip/hip_runtime.h>
__device__ __forceinline__ unsigned ig_tid() { return threadIdx.x; }
__device__ __forceinline__ unsigned ig_nthreads() { return blockDim.x; }
__device__ __forceinline__ unsigned ig_block() { return blockIdx.x; }
__device__ __forceinline__ void ig_barrier_at(int) { __syncthreads(); }
__device__ __forceinline__ unsigned long long ig_clock() { return wall_clock64(); }
__device__ __forceinline__ unsigned ig_shfl_up(unsigned v, unsigned delta) { return __shfl_up(v, delta, 64); }
#define IGD __device__ __forceinline__
#define IGN __device__ __noinline__
#endif

// A device pointer known to address global memory.  Pointers that kernels
// read out of descriptors are generic, so their accesses compile to flat
// instructions, which also count against the LDS wait counter: every LDS
// wait after them would wait for global memory too.  gmem(p)[i] compiles to
// global loads and stores instead.
#ifdef IG_HOST_SIM
template <class T>
inline T* gmem(T* p) {
    return p;
}
template <class T>
inline T ig_load_agent(const T* p) {
    return __atomic_load_n(p, __ATOMIC_SEQ_CST);
}
#else
// A load that reads the level-2 cache, where atomics are performed, not a
// possibly older copy in the compute unit's level-1 cache.
template <class T>
__device__ __forceinline__ T ig_load_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
#endif

// Global-memory pointers in the kernels' device code: descriptors hold their
// arrays as global-address-space pointers, so that accesses compile to
// global (not flat) instructions, which do not count against the LDS wait
// counter.  Host code (and translation units without kernels, which set no
// IG_KERNEL_TU) sees plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__) && defined(IG_KERNEL_TU)
#define IG_G __attribute__((address_space(1)))
#else
#define IG_G
#endif

namespace igd {

typedef uint8_t u8;
typedef uint16_t u16;
typedef uint32_t u32;
typedef unsigned long long u64;
typedef int64_t i64;
typedef int32_t i32;

constexpr u32 NONE = 0xFFFFFFFFu;
constexpr u32 MAX_BUF = IG_MAX_BUFFERS;
constexpr u32 MAX_LIVE = 16;   // live allocations per (buffer, memory)
constexpr u32 MAX_PLAN = 16;   // planned boxes per (buffer, memory) while the queue is non-empty
constexpr u32 MAX_THREADS = 1024;
constexpr u32 MAX_CHUNKS = 4096;
constexpr u32 RB_SLOTS = 7;    // reader ids per reader block (+1 word: next)
constexpr u32 RD_CACHE = 4;    // accesses per kernel whose read scans can be shared
constexpr u32 MAX_BIG = 4;     // large coherence reads per memory and task scanned by a thread team
constexpr u32 BIG_CELLS = 512; // grid cells from which a read region is scanned by a team

enum CmdKind : u32 { CMD_BUFFER = 1, CMD_TASK = 2, CMD_EPOCH = 3, CMD_DESTROY = 4, CMD_SHUTDOWN = 5 };

// One recorded command (host-written, device-read).
struct DevCmd {
    u32 kind;
    u32 arg;        // buffer id (BUFFER, DESTROY) or task id (TASK)
    u32 dims;       // BUFFER
    u32 elem_size;  // BUFFER
    u32 init;       // BUFFER
    u32 pad[3];
    i64 ext[3];       // BUFFER
    ig_task_desc task;  // TASK
};

// Per-buffer grid and map arrays (offsets are word offsets into the heap).
struct DBuf {
    u32 alive, dims, init, user_alloc;
    i64 ext[3];
    u32 n[3];       // cells per dimension
    u32 bp_off[3];  // i64[n[d]+1] breakpoints
    u32 hx_off[3];  // open-addressing hash: coordinate -> breakpoint index (i64 key, u32 value, 4 words a slot)
    u32 hx_bits[3]; // log2 of the slot count
    u32 ncells;
    u32 prod_off;   // u32[ncells]   original producer (NONE: uninitialised)
    u32 pm_off;     // u32[ncells]   producer memory
    u32 mask_off;   // u64[ncells*mw] up-to-date memories
    u32 init_off;   // u32[ncells]   initialised (Sec. 4.4)
    u32 uninit;     // cells not yet initialised (0: the whole buffer is)
    u32 stamp_off;  // u64[ncells]   overlapping-write detection: (task+1)<<32 | chunk
    u32 wcp_off;    // u32[ncells]   task graph (horizon mode 1): critical-path length of the last writer task
    u32 rcp_off;    // u32[ncells]   the longest among the reader tasks since (<= cp_epoch: none)
};

struct DAlloc {
    u32 buffer, mem, alive, ncells;
    i64 lo[3], hi[3];   // allocation box (buffer coordinates)
    u32 clo[3], chi[3]; // the same box in grid cells
    u32 am_off;         // AmCell[ncells]: the allocation map, one 16-byte record per grid cell
    u32 old_am;         // scratch for grid refinement
};

// One cell of an allocation map (Sec. 3.2/3.3 tracking): last writer, with
// bit 31 set when the writer is the allocation's ALLOC; two inline readers;
// the head of an overflow list of reader blocks for further readers.
struct AmCell {
    u32 w, r0, r1, ov;
};
constexpr u32 W_ALLOC = 0x80000000u;

// One region of one (chunk, access) of the task being analysed.
struct Region {
    i64 lo[3], hi[3];
    u32 clo[3], chi[3];
    u32 buffer;
    u32 mode;
    u32 empty;
    u32 pad;
};

// Consecutive kernels of one device with a pure read of the same cells.
struct RdGroup {
    u32 alloc, first, n, nsrc;
    u32 clo[3], chi[3];
};

// A coherence copy found in the counting pass.
struct CopyRec {
    u32 chunk, buffer, src_alloc, dst_alloc;
    u32 src_mem, dst_mem, pad0, pad1;  // pad0: chunk * IG_MAX_ACCESS + access; pad1: instruction offset
                                       // within its device's copies (emission)
    u32 clo[3], chi[3];
};

// A read of a source allocation by a copy, routed to the owner of its memory.
struct InboxRec {
    u32 alloc, reader;
    u32 clo[3], chi[3];
};

// Scalars persisted between launches (mirrored in LDS while a launch runs).
struct Scalars {
    u64 n_instr, n_edges, n_binds;
    u64 warnings, rejected, resizes;
    u32 cmd_next;        // next recorded command to analyse
    u32 n_tasks;         // tasks analysed so far
    u32 next_alloc;      // next allocation id
    u32 S;               // synchronisation point: latest epoch or applied horizon
    u32 E;               // latest epoch
    u32 pending;         // emitted, not yet applied horizon (NONE)
    u32 last_sync;       // latest horizon or epoch (the front starts there)
    u32 tasks_since_sync;
    u32 h;               // horizons queued since the last allocating command
    u32 qlen;            // commands in the lookahead queue
    u32 n_buffers;
    u32 finished;
    u32 heap_top;        // words
    u32 rb_top;          // reader blocks
    i32 error;
    u32 done_tasks;      // leading tasks whose records are complete (none held in the queue)
    u32 cap_what;        // with IG_E_CAPACITY: which capacity (IG_CAP_*)
    // task graph (horizon mode 1): critical-path lengths of the task-level
    // sync point (latest epoch or applied horizon), of the latest epoch, of
    // the generated horizon not yet applied (0: none), the longest path so
    // far and its length at the last horizon or epoch
    u32 cp_sync, cp_epoch, cp_pending, cp_max, cp_last;
    u32 pad;
};

struct DevCtx {
    // --- configuration ---
    u32 nodes, devices, chunks, per_dev, n_dev, n_mem, mw;
    u32 horizon_step, lookahead, flush_horizons, queue_cap;
    u32 threads, n_workers;
    u32 horizon_mode, horizon_max_tasks;
    u32 staging, pad_staging;  // 1: device-to-device copies within a node staged through M1
    u32 cap_cmds, cap_allocs, cap_queue, cap_heap, cap_rb, cap_unit, cap_scr, cap_src, cap_box;
    u32 pad0;
    u64 cap_instr, cap_edges, cap_binds;
    u32 cmd_end;  // commands recorded (set by the host before a launch)
    u32 pad1;
    // --- command log ---
    IG_G DevCmd* cmds;
    // --- outputs (structure of arrays) ---
    IG_G u8* i_kind;
    IG_G u8* i_flags;
    IG_G u16* i_mem;
    IG_G u16* i_src_mem;
    IG_G u32* i_task;
    IG_G u32* i_chunk;
    IG_G u32* i_buffer;
    IG_G u32* i_alloc;
    IG_G u32* i_src_alloc;
    IG_G i64* i_box;  // [6][cap_instr]: min0 min1 min2 max0 max1 max2
    IG_G u32* e_from;
    IG_G u32* e_to;
    IG_G u8* e_kinds;
    IG_G u32* b_instr;
    IG_G u32* b_access;
    IG_G u32* b_alloc;
    IG_G u8* has_succ;
    IG_G i32* task_status;
    IG_G u64* task_t0;   // [cap_cmds] device clock when the task's intake began
    IG_G u64* task_tq;   // [cap_cmds] device clock when its intake ended (compiled at once or queued)
    IG_G u64* task_tc;   // [cap_cmds] device clock when its compilation began
    IG_G u64* task_t1;   // [cap_cmds] device clock when its records were complete
    IG_G u64* phase;     // [32] device-clock ticks per analysis phase (profiling builds only)
    // --- state ---
    IG_G DBuf* bufs;       // [MAX_BUF]
    IG_G DAlloc* allocs;   // [cap_allocs]
    IG_G u32* live_n;      // [MAX_BUF * n_mem]
    IG_G u32* live;        // [MAX_BUF * n_mem * MAX_LIVE]
    IG_G u32* plan_n;      // [MAX_BUF * n_mem]  NONE: not planned (use live)
    IG_G i64* plan;        // [MAX_BUF * n_mem * MAX_PLAN * 6]
    IG_G u32* queue;       // [cap_queue] command index, top bit: horizon
    IG_G u32* heap;        // [cap_heap] words
    IG_G u32* heap_free;   // [32] free-list heads per size class
    IG_G u32* rb;          // [cap_rb * 8] reader blocks
    IG_G u64* rb_free;         // [n_mem] free reader blocks per memory: tag << 32 | head
    // --- per-command scratch ---
    IG_G Region* reg;          // [MAX_CHUNKS * IG_MAX_ACCESS]
    IG_G i64* chunk_lo;        // [MAX_CHUNKS]
    IG_G i64* chunk_hi;        // [MAX_CHUNKS]
    IG_G u32* cons_off;        // [MAX_CHUNKS * IG_MAX_ACCESS]
    IG_G u32* cons_cnt;        // [MAX_CHUNKS * IG_MAX_ACCESS]
    IG_G u32* cons_x;          // [MAX_CHUNKS * IG_MAX_ACCESS] first copy of (chunk, access) within its device
    IG_G u32* k_rank;          // [MAX_CHUNKS] kernel index of a chunk within its device (NONE: empty)
    IG_G u32* big_n;           // [n_mem] large coherence reads deferred to the team scan
    IG_G u32* big_idx;         // [n_mem * MAX_BIG] their (chunk * IG_MAX_ACCESS + access)
    IG_G u32* tm;              // [n_mem * 4] words a thread team shares (offsets, totals, flags)
    IG_G CopyRec* copies;      // [cap_unit]
    IG_G u32* dev_cnt;         // [n_dev] copies per device, then kernels per device
    IG_G u32* dev_base;        // [n_dev]
    IG_G u32* kdev_cnt;        // [n_dev]
    IG_G u32* kdev_base;       // [n_dev]
    IG_G u32* inbox_cnt;       // [n_mem]
    IG_G u32* inbox_off;       // [n_mem]
    IG_G u32* inbox_cur;       // [n_mem]
    IG_G InboxRec* inbox;      // [cap_unit]
    IG_G u32* tab_off;         // [cap_unit] staged edges of each instruction of the unit
    IG_G u32* tab_cnt;         // [cap_unit]
    IG_G u32* stage_from;      // [cap_unit * 4]
    IG_G u8* stage_kind;       // [cap_unit * 4]
    IG_G u32* pair_flag;       // [MAX_BUF * n_mem] (allocation phase)
    IG_G u32* pair_cnt;        // [MAX_BUF * n_mem]
    IG_G u32* pair_acnt;       // [MAX_BUF * n_mem]
    IG_G u32* miss_n;          // [1]
    IG_G i64* miss_val;        // [cap_scr]
    IG_G u32* miss_bd;         // [cap_scr] buffer*4+dim
    IG_G u32* remap;           // [3 * cap_scr] old cell of new cell, per dim
    // --- per-worker scratch ---
    IG_G u64* wk_key;   // [n_workers * cap_scr]
    IG_G u32* wk_val;   // [n_workers * cap_scr]
    IG_G u64* wk_key2;  // [n_workers * cap_scr]
    IG_G u32* wk_val2;  // [n_workers * cap_scr]
    IG_G u64* wk_rsrc;  // [n_workers * RD_CACHE * cap_src] sources of shared read scans
    IG_G RdGroup* wk_grp;  // [n_workers * RD_CACHE] read groups
    IG_G u64* wk_src;   // [threads * cap_src]
    IG_G u64* wk_src2;  // [threads * cap_src]
    IG_G i64* wk_box;   // [n_workers * cap_box * 6]
    // --- persistent scalars ---
    Scalars s;
};

// Per-launch results of the digest/statistics kernel.
struct DevStats {
    unsigned long long digest[3];
    unsigned long long per_kind[8];
    unsigned long long per_dep[5];
};

// What the engine knows of an instruction's dependencies, kept current as
// they are assigned and complete: how many are not yet assigned (unasg), how
// many are incomplete on lanes outside its class (foreign), and of those
// incomplete on its class's lanes the count (inc), the sum of their lanes
// (suml) and of the squares (all on one lane exactly when count * squares
// == sum^2).  Two pairs share a 64-bit word each, so one atomic addition
// updates both (no field ever leaves [0, 2^32), so no carry crosses halves).
struct OooCnt {
    u64 uf;     // unasg | foreign << 32
    u64 is;     // inc | suml << 32
    u64 sumsq;
};
// Per instruction while it is in flight: the next instruction on its lane
// and that one's end, and its own successor list (offset, length).
struct OooRec {
    u32 next, o0, deg, pad;
    u64 next_end;
};

// One graph of an out-of-order engine simulation (ig_ooo.hip).
struct OooGraph {
    // records of the context (device arrays)
    const u8* kind;
    const u8* flags;
    const u16* mem;
    const i64* box;   // [6][box_stride]
    const u32* e_from;
    const u32* e_to;
    u64 box_stride;
    u32 n, ne;
    // results
    ig_ooo_slot* out;     // [n]
    ig_ooo_summary* sum;  // [1]
    i32* status;          // [1]
    // workspace
    u32* out_off;  // [n + 1] successor list offsets (counts before the scan)
    u32* out_adj;  // [ne] successors
    OooCnt* cnt;   // [n] dependency state
    OooRec* rec;   // [n] lane FIFO links and successor ranges (fill cursors during preparation)
    u32* cls;      // [n] lane class
    u64* dur;      // [n]
};

}  // namespace igd

// Launch glue implemented next to the kernels (ig_kernels.hip).
namespace igrt {
int dev_malloc(void** p, size_t bytes);
int dev_free(void* p);
int host_malloc_pinned(void** p, size_t bytes);
int host_free_pinned(void* p);
int copy_h2d(void* dst, const void* src, size_t bytes, void* stream);
int copy_d2h(void* dst, const void* src, size_t bytes, void* stream);
int memset_d(void* dst, int v, size_t bytes, void* stream);
int stream_sync(void* stream);
double clock_khz();
// window: analyse at most this many further commands per context (0: all uploaded)
int launch_analyse(igd::DevCtx* const* dev_ctx_ptrs_device, unsigned n_blocks, unsigned threads, unsigned window,
                   void* stream);
int launch_analyse_wide(igd::DevCtx* const* dev_ctx_ptrs_device, unsigned n_blocks, unsigned threads,
                        unsigned window, void* stream);
int launch_reset(igd::DevCtx* const* dev_ctx_ptrs_device, unsigned n, void* stream);
int launch_gather(igd::DevCtx* const* dev_ctx_ptrs_device, unsigned n, uint64_t* out_dev, void* stream);
// Capture reset + analysis of n contexts as one graph (exec: opaque handle).
int graph_capture(igd::DevCtx* const* dev_ctx_ptrs_device, unsigned n, unsigned threads, void* stream, void** exec);
int graph_launch(void* exec, void* stream);
int graph_destroy(void* exec);
int launch_pack_instructions(const igd::DevCtx* dev_ctx, uint64_t first, uint64_t n, ig_instruction* out_dev,
                             void* stream);
int launch_pack_bindings(const igd::DevCtx* dev_ctx, uint64_t first, uint64_t n, ig_binding* out_dev, void* stream);
int launch_pack_edges(const igd::DevCtx* dev_ctx, uint64_t first, uint64_t n, ig_edge* out_dev, void* stream);
// the out-of-order engine over n_graphs graphs (device array d_graphs); max_n / max_ne size the preparation grids
int launch_ooo(const igd::OooGraph* d_graphs, unsigned n_graphs, uint64_t max_n, uint64_t max_ne, const ig_ooo_params* p,
               void* stream);
int launch_stats(const igd::DevCtx* dev_ctx, uint64_t n_instr, uint64_t n_bind, uint64_t n_edge,
                 igd::DevStats* out_dev, void* stream);
// Events (completion of work queued on a stream) and a side stream.
int event_create(void** ev);
int event_record(void* ev, void* stream);
int event_query(void* ev);  // 1 complete, 0 pending, -1 error
int event_sync(void* ev);
int event_destroy(void* ev);
int stream_create(void** stream);  // non-blocking, default priority
int stream_destroy(void* stream);
// Device address of this GPU's fixed scratch array (IG_NOALLOC_SCRATCH_BYTES),
// looked up once per device on first use; never allocates.
int noalloc_scratch(void** out);
const char* last_error();
}  // namespace igrt
