/*
 * ig_oracle.h -- CPU oracle for instruction-graph generation.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, sequential reference
 * against which the HIP implementation is checked.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never does.  It shares no code and no header with the
 * product (include/ig.h): the record layouts below are written out again on
 * purpose so that both sides can be compared field by field.
 *
 * The oracle follows the paper's description of instruction-graph generation
 * (Sec. 3: work assignment 3.1, allocation 3.2, coherence 3.3, horizons and
 * epochs 3.5; Sec. 4.3 scheduler lookahead; Sec. 4.4 debug checks) on a
 * flattened cluster of integer-id devices.  Every place the paper leaves open
 * is settled by a documented reading; those readings are the definition of
 * parity.
 */
#ifndef IG_ORACLE_H
#define IG_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define IGO_OK 0
#define IGO_W_UNINIT_READ 1
#define IGO_E_INVALID (-1)
#define IGO_E_OVERLAPPING_WRITE (-2)
#define IGO_E_CAPACITY (-3)

/* instruction kinds (Table 1 subset) */
#define IGO_ALLOC 1
#define IGO_COPY 2
#define IGO_FREE 3
#define IGO_KERNEL 4
#define IGO_HORIZON 5
#define IGO_EPOCH 6

/* instruction flags */
#define IGO_F_RESIZE 1
#define IGO_F_INTER_NODE 2

/* edge kind bits */
#define IGO_DEP_TRUE 1
#define IGO_DEP_ANTI 2
#define IGO_DEP_OUTPUT 4
#define IGO_DEP_LIFETIME 8
#define IGO_DEP_SYNC 16

/* access modes, mappers, init */
#define IGO_READ 1
#define IGO_WRITE 2
#define IGO_READ_WRITE 3
#define IGO_MAP_ONE_TO_ONE 0
#define IGO_MAP_NEIGHBORHOOD 1
#define IGO_MAP_ALL 2
#define IGO_MAP_SLICE 3
#define IGO_MAP_FIXED 4
#define IGO_INIT_NONE 0
#define IGO_INIT_HOST 1

#define IGO_MAX_ACCESS 8
#define IGO_NONE32 0xFFFFFFFFu
#define IGO_NONE16 0xFFFFu

typedef struct igo_box {
    int64_t min[3];
    int64_t max[3];
} igo_box;

typedef struct igo_access {
    uint32_t buffer;
    uint8_t mode;
    uint8_t mapper;
    uint8_t slice_dim;
    uint8_t pad;
    int64_t radius[3];
    igo_box fixed;
} igo_access;

typedef struct igo_task_desc {
    uint32_t dims;
    uint32_t n_access;
    igo_box box;
    igo_access access[IGO_MAX_ACCESS];
} igo_task_desc;

typedef struct igo_context_desc {
    uint32_t nodes;
    uint32_t devices_per_node;
    uint32_t chunks;          /* 0: nodes * devices_per_node */
    uint32_t horizon_step;    /* 0: 4 */
    uint32_t lookahead;       /* 0 off, 1 on */
    uint32_t flush_horizons;  /* 0: 2 */
    uint32_t queue_cap;       /* 0: unbounded */
    /* Sec. 3.5: when a horizon enters the command stream.  0: after every
     * horizon_step accepted tasks since the last horizon or epoch.  1: from
     * the task graph -- when its critical-path length has grown by
     * horizon_step since the last horizon or epoch, or when
     * horizon_max_tasks tasks have been accepted since then (0: 16 x
     * horizon_step), whichever comes first. */
    uint32_t horizon_mode;
    uint32_t horizon_max_tasks;
    /* Sec. 3.3, last paragraph: 1 when devices cannot copy to each other
     * directly.  A coherence copy between two devices of one node is then
     * staged through pinned host memory M1 as two copies: device to M1 (it
     * reads the source allocation) and M1 to device (it writes the
     * destination allocation and depends on the first); the staging space is
     * the executor's, outside the graph (allocation id 0 on the M1 side).
     * Copies between nodes are unchanged. */
    uint32_t staging;
} igo_context_desc;

typedef struct igo_instruction {
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
    igo_box box;
} igo_instruction; /* 96 bytes */

typedef struct igo_binding {
    uint64_t instr;
    uint32_t access;
    uint32_t pad;
    uint64_t alloc;
} igo_binding; /* 24 bytes */

typedef struct igo_edge {
    uint64_t from;
    uint64_t to;
    uint32_t kinds;
    uint32_t pad;
} igo_edge; /* 24 bytes */

typedef struct igo_stats {
    uint64_t n_instructions;
    uint64_t n_bindings;
    uint64_t n_edges;
    uint64_t per_kind[8];      /* index = instruction kind */
    uint64_t per_dep[5];       /* edges carrying TRUE, ANTI, OUTPUT, LIFETIME, SYNC */
    uint64_t resizes;          /* allocations replaced by a larger one */
    uint64_t warnings;         /* tasks with an uninitialised read */
    uint64_t tasks_submitted;
    uint64_t tasks_rejected;
    uint64_t digest_instructions;
    uint64_t digest_bindings;
    uint64_t digest_edges;
    /* Terms of the algorithmic-bytes model of the measurement (one count per
     * access, independent of how an implementation fragments its maps):
     *   u_w        allocation-map writer updates: one per ALLOC (its whole
     *              box) and per write access of a COPY or KERNEL (Sec. 3.2)
     *   u_r        allocation-map reader insertions: one per read access of a
     *              COPY or KERNEL
     *   u_b        buffer-map updates: one per coherence COPY (its box joins
     *              the destination's up-to-date memories, Sec. 3.3) and per
     *              KERNEL write (new original producer)
     *   map_boxes  range-mapper evaluations: non-empty chunks x accessors of
     *              every structurally valid task (Sec. 2.1, Sec. 3.1) */
    uint64_t u_w;
    uint64_t u_r;
    uint64_t u_b;
    uint64_t map_boxes;
} igo_stats;

/* One entry of the command trace: every call that reaches the command stream
 * (buffer creation, task, the horizon the stream inserts, epoch, buffer
 * destruction, shutdown), in call order.  Tests use it to check the Sec. 4.3
 * queue decisions (the allocating predicate and the moment each command is
 * compiled) against an independent brute force. */
#define IGO_EV_BUFFER 1
#define IGO_EV_TASK 2      /* accepted task, pushed to the command queue */
#define IGO_EV_REJECTED 3  /* task rejected by the Sec. 4.4 overlap check */
#define IGO_EV_HORIZON 4
#define IGO_EV_EPOCH 5
#define IGO_EV_DESTROY 6
#define IGO_EV_SHUTDOWN 7
typedef struct igo_event {
    uint32_t kind;         /* IGO_EV_* */
    uint32_t arg;          /* buffer id (BUFFER, DESTROY), task id (TASK, REJECTED), else NONE */
    uint32_t allocating;   /* TASK with lookahead on: the allocating predicate at push time */
    uint32_t compiled_at;  /* TASK, HORIZON: index of the event during which it was compiled */
    uint64_t n_instr;      /* instructions emitted when the event began */
} igo_event; /* 24 bytes */

typedef struct igo_context igo_context;

int32_t igo_context_create(const igo_context_desc* desc, igo_context** out);
int32_t igo_context_destroy(igo_context* ctx);
int32_t igo_buffer_create(igo_context* ctx, uint32_t dims, const int64_t extent[3],
                          uint32_t elem_size, uint32_t init, uint32_t* out_buffer);
int32_t igo_buffer_destroy(igo_context* ctx, uint32_t buffer);
int32_t igo_submit_task(igo_context* ctx, const igo_task_desc* task, uint64_t* out_task);
int32_t igo_epoch(igo_context* ctx);
int32_t igo_shutdown(igo_context* ctx);
int32_t igo_flush_window(igo_context* ctx);
int32_t igo_counts(igo_context* ctx, uint64_t* n_instr, uint64_t* n_bind, uint64_t* n_edge,
                   uint64_t* n_tasks);
int32_t igo_fetch_instructions(igo_context* ctx, igo_instruction* dst, size_t cap, size_t* n_out);
int32_t igo_fetch_bindings(igo_context* ctx, igo_binding* dst, size_t cap, size_t* n_out);
int32_t igo_fetch_edges(igo_context* ctx, igo_edge* dst, size_t cap, size_t* n_out);
int32_t igo_fetch_task_status(igo_context* ctx, int32_t* dst, size_t cap, size_t* n_out);
int32_t igo_stats_get(igo_context* ctx, igo_stats* out);
int32_t igo_fetch_events(igo_context* ctx, igo_event* dst, size_t cap, size_t* n_out);
size_t igo_event_count(igo_context* ctx);

/* box-set primitives, exported so that tests can pin them against brute force */
size_t igo_box_subtract(const igo_box* a, const igo_box* b, igo_box* out /* >= 6 */);
int32_t igo_box_merges(const igo_box* a, const igo_box* b);
size_t igo_canonical(const igo_box* in, size_t n, igo_box* out, size_t cap);
size_t igo_merge_fixpoint(const igo_box* in, size_t n, igo_box* out, size_t cap);
/* chunk split and range mapping, exported for the same reason */
int32_t igo_split(uint32_t nodes, uint32_t devices, uint32_t chunks, const igo_box* task,
                  igo_box* out_chunks /* chunks */);
int32_t igo_map(const igo_access* acc, uint32_t task_dims, const igo_box* chunk,
                uint32_t buf_dims, const int64_t extent[3], igo_box* out);
uint64_t igo_digest(const uint64_t* words, size_t n_records, size_t words_per_record);

/* ---------------------------------------------------------------------------
 * Out-of-order engine (Sec. 4.1), simulated over a finished instruction
 * graph.  Lanes are in-order queues: lanes_per_device per device (device
 * memory 2 + d) for its kernels and the copies into it, and host_lanes for
 * allocations, frees and copies into host memory; horizons and epochs
 * complete in the engine itself when their dependencies have.  Time is
 * integer nanoseconds.  At each moment the engine makes rounds over the
 * unassigned instructions whose ids lie within `window` of the first
 * unassigned one: a round takes every one that is assignable at its start,
 * in id order -- directly when all its dependencies are complete (to the
 * lane of its class that frees up first, lowest number on ties), or, with
 * `eager`, eagerly when every incomplete dependency is issued to one and
 * the same lane of its class (behind them, which the lane's order makes
 * safe).  When a round takes none, time moves to the next completion.
 * --------------------------------------------------------------------------- */
typedef struct igo_ooo_params {
    uint32_t devices;            /* device memories 2 .. devices + 1 */
    uint32_t lanes_per_device;   /* >= 1 */
    uint32_t host_lanes;         /* >= 1 */
    uint32_t window;             /* >= 1 */
    uint32_t eager;              /* 0 or 1 */
    uint32_t pad;
    uint64_t kernel_ns;          /* KERNEL: kernel_ns + volume * kernel_ns_per_kelem / 1024 */
    uint64_t kernel_ns_per_kelem;
    uint64_t copy_ns;            /* COPY: copy_ns + volume * copy_ns_per_kelem / 1024 (+ inter_node_ns) */
    uint64_t copy_ns_per_kelem;
    uint64_t inter_node_ns;
    uint64_t alloc_ns;
    uint64_t free_ns;
} igo_ooo_params;

#define IGO_OOO_ENGINE 0u  /* horizon / epoch: completed by the engine */
#define IGO_OOO_DIRECT 1u
#define IGO_OOO_EAGER 2u

typedef struct igo_ooo_slot {
    uint32_t lane;   /* IGO_NONE32 for the engine's own instructions */
    uint32_t how;    /* IGO_OOO_* */
    uint64_t issue;  /* the moment it was assigned */
    uint64_t start;
    uint64_t end;
} igo_ooo_slot; /* 32 bytes */

typedef struct igo_ooo_summary {
    uint64_t makespan;
    uint64_t direct, eager;
    uint64_t steps;   /* moments at which rounds ran */
    uint64_t rounds;
} igo_ooo_summary;

/* ins[i].id must be i; edges in any order with from < to.  Returns
 * IGO_E_INVALID on bad arguments or an instruction whose memory has no
 * lane. */
int32_t igo_ooo_simulate(const igo_instruction* ins, size_t n, const igo_edge* edges, size_t n_edges,
                         const igo_ooo_params* p, igo_ooo_slot* out, igo_ooo_summary* sum);

#ifdef __cplusplus
}
#endif
#endif
