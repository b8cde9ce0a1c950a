/*
 * ig.h -- C ABI of the MI355X instruction-graph generator (libig).
 *
 * Instruction-graph (IDAG) generation after Knorr, Salzmann, Thoman and
 * Fahringer, "Concurrent Scheduling of High-Level Parallel Programs on
 * Multi-GPU Systems" (arXiv 2503.10516): a stream of data-parallel tasks with
 * range-mapped buffer accesses is split over a simulated cluster of
 * integer-id devices (Sec. 3.1) and compiled into allocations and resizes
 * (Sec. 3.2), coherence copies with producer and consumer split (Sec. 3.3),
 * device kernels, horizons and epochs (Sec. 3.5, Table 1), with true, anti,
 * output, allocation-lifetime and synchronisation edges (legend of the IDAG
 * figure, Sec. 3.6), under the scheduler lookahead of Sec. 4.3 and the debug
 * checks of Sec. 4.4.
 *
 * All analysis runs in HIP kernels on one gfx950 GPU, one workgroup per
 * stream; the host side only validates arguments, records commands and moves
 * records.  Nothing here is executed on the simulated devices.
 *
 * Conventions
 *   - Every entry point returns an ig_status: 0 = IG_OK, 1 = IG_W_UNINIT_READ
 *     (only as a per-task status), negative = error.  An error leaves the
 *     context unchanged.
 *   - Device memory: the caller may hand in an arena (device pointer + size,
 *     e.g. a torch tensor) that must outlive the context; with arena == NULL
 *     the library allocates (and frees) its own.  ig_arena_bytes() gives the
 *     size a descriptor needs.  The stream (hipStream_t, may be NULL = the
 *     default stream) is the caller's; all work of a context is ordered on it.
 *   - Descriptors are copied; the caller may free them on return.
 *   - Threading: one host thread per context at a time; contexts are
 *     independent.  Ids (instructions, allocations, tasks) are per context,
 *     so a stream's output is the same alone and batched with others.
 *   - Submission is asynchronous: ig_submit_task validates and records; the
 *     analysis of everything recorded runs at ig_flush_window (asynchronously
 *     on the stream) and its per-task status (0, IG_W_UNINIT_READ or
 *     IG_E_OVERLAPPING_WRITE) is read with ig_fetch_task_status after
 *     ig_sync.
 */
#ifndef IG_H
#define IG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ig_status;

#define IG_OK 0
#define IG_W_UNINIT_READ 1           /* Sec. 4.4: read of uninitialised data (task accepted) */
#define IG_E_INVALID (-1)            /* bad argument, unknown buffer, mapper/dimension mismatch */
#define IG_E_OVERLAPPING_WRITE (-2)  /* Sec. 4.4: chunks of one task write overlapping regions */
#define IG_E_CAPACITY (-3)           /* a device-side table or the arena is too small */
#define IG_E_DEVICE (-4)             /* a HIP runtime error */
#define IG_E_BUSY (-5)               /* serving admission: no free slot or arena memory */
#define IG_E_INTERNAL (-6)           /* an invariant of the analysis state failed (a library bug) */

/* Which capacity an IG_E_CAPACITY raised during analysis ran out of
 * (ig_stats.capacity_exceeded, ig_progress.capacity_exceeded). */
#define IG_CAP_INSTRUCTIONS 1  /* cap_instructions */
#define IG_CAP_EDGES 2         /* cap_edges */
#define IG_CAP_BINDINGS 3      /* bindings (2 x cap_instructions) */
#define IG_CAP_STATE 4         /* cap_state_words: cell grids and allocation maps */
#define IG_CAP_READERS 5       /* reader-list blocks (cap_state_words / 4 blocks of 8 words) */
#define IG_CAP_UNIT 6          /* cap_unit: instructions or staged edges of one compile unit */
#define IG_CAP_SCRATCH 7       /* fixed per-worker scratch (boxes, grid coordinates, sources) */
#define IG_CAP_LIVE 8          /* live or planned allocations per (memory, buffer) */
#define IG_CAP_COMMANDS 9      /* lookahead queue (2 x cap_commands) */
#define IG_CAP_BUFFERS 10      /* IG_MAX_BUFFERS */
#define IG_CAP_ALLOCS 11       /* allocation ids */

/* instruction kinds (Table 1: the subset on the hot path) */
#define IG_ALLOC 1
#define IG_COPY 2
#define IG_FREE 3
#define IG_KERNEL 4
#define IG_HORIZON 5
#define IG_EPOCH 6

/* instruction flags */
#define IG_F_RESIZE 1      /* copy of a resize chain (Sec. 3.2) */
#define IG_F_INTER_NODE 2  /* copy between devices of different nodes */

/* dependency kinds, a bit set per edge */
#define IG_DEP_TRUE 1
#define IG_DEP_ANTI 2
#define IG_DEP_OUTPUT 4
#define IG_DEP_LIFETIME 8
#define IG_DEP_SYNC 16

/* access modes (bit set), range mappers, buffer initialisation */
#define IG_READ 1
#define IG_WRITE 2
#define IG_READ_WRITE 3
#define IG_MAP_ONE_TO_ONE 0
#define IG_MAP_NEIGHBORHOOD 1
#define IG_MAP_ALL 2
#define IG_MAP_SLICE 3
#define IG_MAP_FIXED 4
#define IG_INIT_NONE 0
#define IG_INIT_HOST 1

#define IG_MAX_ACCESS 8
#define IG_MAX_BUFFERS 64
#define IG_MAX_DEVICES 254
#define IG_NONE32 0xFFFFFFFFu
#define IG_NONE16 0xFFFFu

/* A half-open box [min, max) in up to three dimensions; unused dimensions
 * are [0, 1). */
typedef struct ig_box {
    int64_t min[3];
    int64_t max[3];
} ig_box;

/* One accessor (Sec. 2.1): buffer, mode and range mapper.
 *   one_to_one   region = chunk box
 *   neighborhood region = chunk box grown by radius[d] on both sides
 *   all          region = whole buffer
 *   slice        region = chunk box widened to the buffer in slice_dim
 *   fixed        region = `fixed`
 * Every region is clipped to the buffer.  one_to_one, neighborhood and slice
 * require task dims == buffer dims. */
typedef struct ig_access {
    uint32_t buffer;
    uint8_t mode;
    uint8_t mapper;
    uint8_t slice_dim;
    uint8_t pad;
    int64_t radius[3];
    ig_box fixed;
} ig_access;

/* A task (one command group, one kernel): its index box and accessors. */
typedef struct ig_task_desc {
    uint32_t dims;
    uint32_t n_access;
    ig_box box;
    ig_access access[IG_MAX_ACCESS];
} ig_task_desc;

typedef struct ig_context_desc {
    uint32_t nodes;             /* simulated nodes, >= 1 */
    uint32_t devices_per_node;  /* devices per node, nodes*devices <= 254 */
    uint32_t chunks;            /* chunks per task, a multiple of nodes*devices (0: one per device) */
    uint32_t horizon_step;      /* accepted tasks between horizons (0: 4) */
    uint32_t lookahead;         /* Sec. 4.3 command queue: 0 off, 1 on */
    uint32_t flush_horizons;    /* horizons after the last allocating command before a flush (0: 2) */
    uint32_t queue_cap;         /* flush when the queue holds this many commands (0: unbounded) */
    uint32_t threads;           /* workgroup size of this stream's analysis (0: 256); tuning only */
    uint32_t horizon_mode;      /* Sec. 3.5: 0 a horizon every horizon_step accepted tasks; 1 from the
                                   task graph: when its critical-path length has grown by horizon_step
                                   since the last horizon or epoch, or horizon_max_tasks tasks came since */
    uint32_t horizon_max_tasks; /* horizon_mode 1: tasks between horizons at most (0: 16 x horizon_step) */
    uint32_t staging;           /* Sec. 3.3, last paragraph: 1 when devices cannot copy to each other: a
                                   coherence copy between two devices of one node becomes a copy into
                                   pinned host memory M1 (reading the source allocation) and one from it
                                   (writing the destination, depending on the first); the staging space
                                   is the executor's (allocation 0 on the M1 side).  0: direct copies */
    uint32_t pad2;
    uint64_t cap_commands;      /* recorded commands (0: 65536) */
    uint64_t cap_instructions;  /* output instructions (0: 1<<20) */
    uint64_t cap_edges;         /* output edges (0: 4 * cap_instructions) */
    uint64_t cap_state_words;   /* 32-bit words for region maps and grids (0: 1<<24) */
    uint64_t cap_unit;          /* instructions of one compiled command, edges staged x8 (0: 1<<18) */
    uint64_t cap_scratch;       /* per-worker scratch entries: grid coordinates per dimension, stale
                                   cells of one read, sources of one instruction x2, boxes x4 (0: 8192) */
    void* arena;                /* caller-owned device memory, or NULL */
    uint64_t arena_bytes;
    void* stream;               /* hipStream_t, or NULL */
} ig_context_desc;

/* Output records.  Ids are per context.  For COPY, box is in buffer
 * coordinates; KERNEL: the chunk's index box; ALLOC/FREE: the allocation's
 * box; HORIZON/EPOCH: empty.  Unused ids are IG_NONE32 / IG_NONE16, unused
 * allocation ids 0. */
typedef struct ig_instruction {
    uint64_t id;
    uint8_t kind;
    uint8_t flags;
    uint16_t mem;
    uint16_t src_mem;
    uint16_t pad0;
    uint32_t task;
    uint32_t chunk;
    uint32_t buffer;
    uint32_t pad1;
    uint64_t alloc;
    uint64_t src_alloc;
    ig_box box;
} ig_instruction; /* 96 bytes */

/* Which allocation backs access `access` of KERNEL `instr` (0: empty region). */
typedef struct ig_binding {
    uint64_t instr;
    uint32_t access;
    uint32_t pad;
    uint64_t alloc;
} ig_binding; /* 24 bytes */

typedef struct ig_edge {
    uint64_t from;
    uint64_t to;
    uint32_t kinds; /* IG_DEP_* bit set */
    uint32_t pad;
} ig_edge; /* 24 bytes */

typedef struct ig_stats {
    uint64_t n_instructions;
    uint64_t n_bindings;
    uint64_t n_edges;
    uint64_t per_kind[8];
    uint64_t per_dep[5];
    uint64_t resizes;
    uint64_t warnings;
    uint64_t tasks_submitted;
    uint64_t tasks_rejected;
    uint64_t digest_instructions;
    uint64_t digest_bindings;
    uint64_t digest_edges;
    uint64_t commands_analysed;
    uint64_t launches;
    uint64_t state_words_used;    /* high-water mark of the state heap (cap_state_words) */
    uint64_t reader_blocks_used;  /* high-water mark of the reader-list blocks */
    uint64_t capacity_exceeded;   /* IG_CAP_* after an IG_E_CAPACITY, else 0 */
    double phase_us[16];       /* device time per analysis phase (profiling builds; else 0) */
    uint64_t phase_count[16];
} ig_stats;

typedef struct ig_context ig_context;

/* Device memory a descriptor needs (arena size): the command log, the
 * output records and the region maps of the simulated cluster (Sec. 3.2:
 * memories and allocations as numeric ids).  Errors: IG_E_INVALID. */
ig_status ig_arena_bytes(const ig_context_desc* desc, uint64_t* bytes);

/* Create a context: one user program on a simulated cluster of nodes x
 * devices (Sec. 3.1), memory M0 the user's host memory, M1 pinned host
 * memory and M2.. the devices (Sec. 3.2).  Validates the cluster shape,
 * prepares device state and records the initial epoch I0 (Sec. 2.4,
 * Table 1).  Errors: IG_E_INVALID, IG_E_CAPACITY (arena too small),
 * IG_E_DEVICE. */
ig_status ig_context_create(const ig_context_desc* desc, ig_context** out);

/* Destroy: waits for outstanding work on the context's stream; frees
 * library-owned memory.  (The program's end is ig_shutdown, Sec. 3.2.) */
ig_status ig_context_destroy(ig_context* ctx);

/* Record a buffer (ids 0, 1, ... in creation order).  IG_INIT_HOST buffers
 * are up to date in user memory M0 (Sec. 3.2).  Errors: IG_E_INVALID,
 * IG_E_CAPACITY (more than IG_MAX_BUFFERS). */
ig_status ig_buffer_create(ig_context* ctx, uint32_t dims, const int64_t extent[3], uint32_t elem_size,
                           uint32_t init, uint32_t* out_buffer);

/* Record the destruction of a buffer: flushes the command queue, then frees
 * its device allocations (Sec. 3.2).  Errors: IG_E_INVALID. */
ig_status ig_buffer_destroy(ig_context* ctx, uint32_t buffer);

/* Record one task; *out_task receives its id.  Structural errors
 * (IG_E_INVALID, IG_E_CAPACITY) are returned here; the Sec. 4.4 outcome is
 * the task's status after analysis. */
ig_status ig_submit_task(ig_context* ctx, const ig_task_desc* task, uint64_t* out_task);

/* Record n tasks at once (ids out_first, out_first+1, ...).  Stops at the
 * first invalid descriptor, recording the ones before it. */
ig_status ig_submit_tasks(ig_context* ctx, const ig_task_desc* tasks, size_t n, uint64_t* out_first);

/* Record a user epoch: flush the queue, then synchronise (Table 1). */
ig_status ig_epoch(ig_context* ctx);

/* Record shutdown: destroy every remaining buffer (their allocations are
 * freed, Sec. 3.2), then the final epoch (Table 1).  No command may follow. */
ig_status ig_shutdown(ig_context* ctx);

/* Analyse everything recorded so far (asynchronously on the stream):
 * commands enter the lookahead queue or are compiled into instructions
 * (Sec. 3, Sec. 4.3).  Does not force a lookahead flush: output never
 * depends on timing. */
ig_status ig_flush_window(ig_context* ctx);

/* Analyse the pending windows of n contexts in ONE launch (one workgroup
 * per context; all must use the same `threads`); each context's graph is
 * the one ig_flush_window gives (Sec. 3).  stream: NULL = the first
 * context's stream. */
ig_status ig_batch_flush(ig_context* const* ctxs, size_t n, void* stream);

/* As ig_batch_flush, but each context analyses at most max_commands further
 * recorded commands in this launch (0: all); later launches continue where
 * it stopped.  Bounds the duration of one launch; the output is the same
 * for every window. */
ig_status ig_batch_flush_window(ig_context* const* ctxs, size_t n, void* stream, uint32_t max_commands);

/* Forget the analysis results of n contexts (as ig_rewind) with one kernel
 * launch on the stream (NULL = the first context's stream).
 *
 * The batched calls (ig_batch_flush, _window, _rewind, _progress) write the
 * table of context pointers into the first context's staging area and wait
 * for the stream before reusing it.  Errors: IG_E_INVALID (no contexts, a
 * NULL context, or contexts built with different `threads`), IG_E_CAPACITY
 * (more contexts than the staging area holds), IG_E_DEVICE. */
ig_status ig_batch_rewind(ig_context* const* ctxs, size_t n, void* stream);

/* Progress of n contexts, gathered on the device and copied back in one
 * transfer (waits for the stream).  tasks_done: leading tasks whose records
 * are complete, i.e. analysed and not held in the lookahead queue;
 * tasks_seen: tasks analysed (queued or compiled); error: a negative status
 * raised during analysis, else 0; finished: shutdown analysed;
 * commands_done: recorded commands analysed.  out[i] belongs to ctxs[i]. */
typedef struct ig_progress {
    uint64_t tasks_done;
    uint64_t tasks_seen;
    int32_t error;
    uint32_t finished;
    uint32_t capacity_exceeded;  /* IG_CAP_* after an IG_E_CAPACITY, else 0 */
    uint32_t commands_done;      /* recorded commands analysed so far */
} ig_progress;
ig_status ig_batch_progress(ig_context* const* ctxs, size_t n, void* stream, ig_progress* out);

/* As ig_batch_progress, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The context-pointer table and the gathered progress words live
 * in a fixed device array of IG_NOALLOC_SCRATCH_BYTES that every GPU holds
 * once for the life of the process (its address is looked up per device on
 * the first call with that device current), instead of the first context's
 * staging area; the caller's `out` array doubles as the host staging of the
 * table.  Calls nothing that allocates (no hipMalloc/hipFree, no host heap).
 * Every word read back is written by the gather kernel of the same call, so
 * nothing needs clearing between calls.  Calls that overlap on one GPU (from
 * several threads or on several streams) share that array and race; the
 * caller must order them.  Errors: IG_E_INVALID (as ig_batch_progress),
 * IG_E_CAPACITY (n > IG_NOALLOC_MAX_CONTEXTS), IG_E_DEVICE (a HIP error, or
 * a device index >= IG_NOALLOC_MAX_DEVICES). */
#define IG_NOALLOC_MAX_CONTEXTS 4096
#define IG_NOALLOC_MAX_DEVICES 64
#define IG_NOALLOC_SCRATCH_BYTES (IG_NOALLOC_MAX_CONTEXTS * (8 + 32))
ig_status ig_batch_progress_noalloc(ig_context* const* ctxs, size_t n, void* stream, ig_progress* out);

/* A captured batched re-analysis (Sec. 3 graph generation for many streams
 * in one persistent launch): the commands recorded so far are uploaded once;
 * every ig_graph_launch forgets the previous results of all n contexts and
 * analyses their recorded streams from the start, as ig_batch_rewind followed
 * by ig_batch_flush would, as one HIP graph (a reset kernel, then the
 * analysis kernel with one workgroup per context).  The graph owns a small
 * device table of the context pointers; the contexts must outlive it and
 * must not be re-created meanwhile.  Errors: IG_E_INVALID, IG_E_DEVICE. */
typedef struct ig_graph ig_graph;
ig_status ig_batch_graph_create(ig_context* const* ctxs, size_t n, void* stream, ig_graph** out);
ig_status ig_graph_launch(ig_graph* graph, void* stream);
ig_status ig_graph_destroy(ig_graph* graph);

/* ---------------------------------------------------------------------------
 * Serving (continuous batching).  Sessions are independent streams, each in
 * its own context, so a session's records are the same alone and in the mix
 * (ids are per context).  A server holds up to `slots` sessions and a budget
 * of arena bytes; a session is admitted when a slot and its arena bytes are
 * free, recorded into while earlier launches run, and analysed in batched
 * launches over every session with new commands (one workgroup each),
 * queued asynchronously on the server's stream: commands travel through
 * pinned staging, progress comes back through pinned memory and an event,
 * and admission prepares the new context on a side stream, so no call but
 * a waiting poll blocks on the device.
 * --------------------------------------------------------------------------- */
typedef struct ig_server ig_server;

typedef struct ig_server_desc {
    uint32_t slots;         /* sessions held at once, 1..4096 */
    uint32_t threads;       /* workgroup size of every session (0: 256) */
    uint32_t window;        /* commands per session per launch (0: all recorded) */
    uint32_t max_inflight;  /* launches queued on the stream at once, 1..8 (0: 2) */
    uint64_t arena_budget;  /* arena bytes (ig_arena_bytes) all sessions may take together, whoever
                               provides the memory (0: unbounded) */
    uint64_t stage_bytes;   /* pinned staging of commands per launch (0: 8 MiB; at least one command) */
    void* stream;           /* hipStream_t of the launches (NULL: the default stream) */
} ig_server_desc;

/* What a poll reports for one occupied slot (from the latest collected
 * launch that included it). */
typedef struct ig_session_progress {
    uint32_t slot;
    uint32_t in_flight;          /* part of a launch not collected yet */
    uint64_t tasks_done;         /* leading tasks whose records are complete (fetchable) */
    uint64_t tasks_seen;         /* tasks analysed (queued or compiled) */
    int32_t error;               /* a negative status raised during analysis, else 0 */
    uint32_t finished;           /* shutdown analysed */
    uint32_t commands_done;      /* recorded commands analysed */
    uint32_t commands_recorded;  /* recorded commands */
} ig_session_progress; /* 40 bytes */

/* Create / destroy a server.  Destroy waits for the queued launches and
 * destroys the contexts still held.  Errors: IG_E_INVALID, IG_E_DEVICE. */
ig_status ig_server_create(const ig_server_desc* desc, ig_server** out);
ig_status ig_server_destroy(ig_server* srv);

/* Admission: a context for `desc` (its stream is replaced by the server's;
 * desc->threads must equal the server's or be 0) in a free slot.  IG_E_BUSY
 * when every slot is taken or its arena would exceed the budget; the caller
 * polls and tries again.  Errors: IG_E_INVALID, IG_E_DEVICE, IG_E_CAPACITY. */
ig_status ig_server_admit(ig_server* srv, const ig_context_desc* desc, uint32_t* out_slot);

/* The session's context, for the recording calls (ig_buffer_create,
 * ig_buffer_destroy, ig_epoch, ig_shutdown, fetch and stats after it is
 * detached).  Do not call ig_flush_window, ig_sync or ig_rewind on it while
 * it is held by the server.  Errors: IG_E_INVALID (free slot). */
ig_status ig_server_session(ig_server* srv, uint32_t slot, ig_context** out);

/* Record a task into a session (= ig_submit_task on its context). */
ig_status ig_server_submit(ig_server* srv, uint32_t slot, const ig_task_desc* task, uint64_t* out_task);

/* Collect finished launches and queue new ones: every launch whose event
 * has completed is collected (wait != 0: the oldest queued launch is waited
 * for first); then, while fewer than max_inflight launches are queued, one
 * launch covers every session with commands that no queued launch covers
 * (uploading what fits in the staging).  out receives one entry per
 * occupied slot (at most cap); *n_out the number written.  Errors:
 * IG_E_INVALID, IG_E_DEVICE. */
ig_status ig_server_poll(ig_server* srv, uint32_t wait, ig_session_progress* out, size_t cap, size_t* n_out);

/* Detach a session whose launches have been collected: its slot and arena
 * budget are freed, and the context (with its records) passes to the
 * caller, who destroys it with ig_context_destroy.  IG_E_BUSY while a
 * queued launch covers it.  Errors: IG_E_INVALID. */
ig_status ig_server_detach(ig_server* srv, uint32_t slot, ig_context** out);

/* Wait for the context's outstanding work; reports IG_E_CAPACITY,
 * IG_E_INTERNAL or IG_E_DEVICE raised during analysis.  (A host-side wait;
 * the program-level synchronisation is ig_epoch, Sec. 2.4.) */
ig_status ig_sync(ig_context* ctx);

/* Forget all analysis results (the recorded commands stay); the next flush
 * re-analyses the stream from the start, giving the same graph (the
 * analysis is a function of the command stream, Sec. 3).  Used to re-run a
 * recorded stream. */
ig_status ig_rewind(ig_context* ctx);

/* Counts of the IDAG records produced so far (Sec. 3.6): instructions,
 * kernel bindings, edges, and tasks analysed (after ig_sync). */
ig_status ig_counts(ig_context* ctx, uint64_t* n_instr, uint64_t* n_bind, uint64_t* n_edge, uint64_t* n_tasks);

/* Copy records into host arrays, continuing from the previous fetch:
 * instructions in id order, which is a topological order (Sec. 4.1), of the
 * kinds of Table 1 used here; kernel bindings by (instruction, access); edges
 * by (to, from) with the dependency kinds of the IDAG figure's legend
 * (Sec. 3.6); per-task statuses of the Sec. 4.4 checks. */
ig_status ig_fetch_instructions(ig_context* ctx, ig_instruction* dst, size_t cap, size_t* n_out);
ig_status ig_fetch_bindings(ig_context* ctx, ig_binding* dst, size_t cap, size_t* n_out);
ig_status ig_fetch_edges(ig_context* ctx, ig_edge* dst, size_t cap, size_t* n_out);
ig_status ig_fetch_task_status(ig_context* ctx, int32_t* dst, size_t cap, size_t* n_out);

/* Per-task timing from the device clock, in nanoseconds relative to the
 * first task's intake, four values per task i:
 *   dst[4*i+0]  intake began (structural checks, Sec. 4.4 checks)
 *   dst[4*i+1]  intake ended: the task was compiled at once or entered the
 *               lookahead queue (Sec. 4.3)
 *   dst[4*i+2]  its compilation began (after any lookahead holding)
 *   dst[4*i+3]  its records were complete
 * so dst[4*i+2] - dst[4*i+1] is the time the lookahead held the task.  A
 * rejected task has all of the last three equal.  cap = tasks. */
ig_status ig_fetch_task_times(ig_context* ctx, double* dst, size_t cap, size_t* n_out);

/* Per-kind counts (Table 1), per-dependency-kind counts (Sec. 3.6),
 * resizes (Sec. 3.2, 4.3), warnings (Sec. 4.4) and the three record
 * digests, all computed on the device. */
ig_status ig_stats_get(ig_context* ctx, ig_stats* out);

/* ---------------------------------------------------------------------------
 * Out-of-order engine (Sec. 4.1), simulated on the device over finished
 * graphs.  The executor keeps several in-order queues ("lanes") per device
 * for its kernels and the copies into it, and host lanes for allocations,
 * frees and copies into host memory; horizons and epochs complete in the
 * engine itself once their dependencies have.  An instruction is assigned
 * directly when every dependency is complete (to the lane of its class that
 * frees up first, the lowest on ties), or, with `eager`, eagerly when every
 * incomplete dependency sits on one and the same lane of its class, behind
 * which the lane's FIFO order makes it safe.  Time is integer nanoseconds
 * under the cost model below.  At each moment the engine makes rounds over
 * the unassigned instructions whose ids lie within `window` of the first
 * unassigned one; a round takes every one that is assignable at its start,
 * in id order; when a round takes none, time moves to the next completion.
 *
 * One workgroup simulates one graph; a handle simulates several graphs (one
 * per context) in one launch.  The graphs are the contexts' records as they
 * stand at ig_ooo_create (after ig_sync); records analysed afterwards are
 * not seen until the handle is created again.
 * --------------------------------------------------------------------------- */
#define IG_OOO_MAX_WINDOW 4096u
#define IG_OOO_MAX_LANES 1023u  /* devices * lanes_per_device + host_lanes */
#define IG_OOO_ENGINE 0u        /* horizon / epoch: completed by the engine */
#define IG_OOO_DIRECT 1u
#define IG_OOO_EAGER 2u

typedef struct ig_ooo_params {
    uint32_t devices;            /* lanes for device memories 2 .. devices + 1 */
    uint32_t lanes_per_device;   /* >= 1 */
    uint32_t host_lanes;         /* >= 1 */
    uint32_t window;             /* 1 .. IG_OOO_MAX_WINDOW */
    uint32_t eager;              /* 0 or 1 */
    uint32_t pad;
    uint64_t kernel_ns;          /* KERNEL: kernel_ns + volume * kernel_ns_per_kelem / 1024, volume of its box */
    uint64_t kernel_ns_per_kelem;
    uint64_t copy_ns;            /* COPY: copy_ns + volume * copy_ns_per_kelem / 1024, + inter_node_ns */
    uint64_t copy_ns_per_kelem;  /*       when IG_F_INTER_NODE */
    uint64_t inter_node_ns;
    uint64_t alloc_ns;           /* ALLOC */
    uint64_t free_ns;            /* FREE; kernel_ns, copy_ns, alloc_ns and free_ns must be >= 1 */
} ig_ooo_params;

typedef struct ig_ooo_slot {
    uint32_t lane;   /* lane d * lanes_per_device + q for device memory 2 + d; host lanes follow;
                        IG_NONE32 for the engine's own instructions */
    uint32_t how;    /* IG_OOO_* */
    uint64_t issue;  /* the moment it was assigned */
    uint64_t start;
    uint64_t end;
} ig_ooo_slot; /* 32 bytes, one per instruction, in id order */

typedef struct ig_ooo_summary {
    uint64_t makespan;       /* the last end */
    uint64_t direct, eager;  /* assignments of each kind */
    uint64_t steps;          /* moments at which rounds ran */
    uint64_t rounds;         /* rounds that assigned something */
} ig_ooo_summary;

typedef struct ig_ooo ig_ooo;
/* A simulation handle over the graphs of n contexts (synchronises each
 * context's stream to read its record counts).  Allocates device memory for
 * the per-instruction results (32 bytes each) and a workspace of 64 bytes
 * per instruction and 4 per edge.  Errors: IG_E_INVALID (parameters out of range, a context
 * with an analysis error, more than 2^31 - 1 instructions), IG_E_DEVICE. */
ig_status ig_ooo_create(ig_context* const* ctxs, size_t n, const ig_ooo_params* p, ig_ooo** out);
/* Queue the simulation of every graph on `stream` (asynchronous). */
ig_status ig_ooo_run(ig_ooo* o, void* stream);
/* Device address and length of graph i's results (owned by the handle,
 * valid until ig_ooo_destroy, complete once the run's stream has reached
 * them). */
ig_status ig_ooo_slots(ig_ooo* o, size_t i, ig_ooo_slot** d_slots, uint64_t* n);
/* Wait for the last run and copy graph i's results (up to cap) and summary
 * (may be NULL) to the host.  Returns the graph's status: IG_E_INVALID for a
 * record the engine has no lane for (a device memory beyond `devices`). */
ig_status ig_ooo_fetch(ig_ooo* o, size_t i, ig_ooo_slot* dst, size_t cap, size_t* n_out, ig_ooo_summary* sum);
ig_status ig_ooo_destroy(ig_ooo* o);

const char* ig_status_str(ig_status st);

/* The message of the last HIP runtime error this thread's calls saw (the
 * cause of an IG_E_DEVICE); "" if none.  Owned by the library. */
const char* ig_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
