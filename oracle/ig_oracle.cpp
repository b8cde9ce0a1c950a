/*
 * ig_oracle.cpp -- CPU oracle for instruction-graph generation.
 *
 * TEST INFRASTRUCTURE ONLY: see ig_oracle.h.  Plain sequential C++17, written
 * for readability rather than speed: region maps are flat vectors of disjoint
 * boxes, every query is a linear scan, and every step follows the order in
 * which the paper describes it.
 *
 * Paper passages followed (section / table / listing):
 *   instruction kinds ............... Table 1
 *   hierarchical work assignment .... Sec. 3.1 (split over nodes, then devices)
 *   allocations, resizes, frees ..... Sec. 3.2
 *   coherence, producer split ....... Sec. 3.3
 *   horizons and epochs ............. Sec. 2.4 and Sec. 3.5
 *   dependency kinds ................ caption of the TDAG/CDAG figure and the
 *                                     legend of the IDAG figure (Sec. 3.6)
 *   topological emission order ...... Sec. 4.1
 *   lookahead / command queue ....... Sec. 4.3
 *   out-of-order engine (simulated) . Sec. 4.1 (direct and eager assignment
 *                                     to in-order lanes)
 *   uninitialised-read and
 *   overlapping-write detection ..... Sec. 4.4
 * The readings that settle what the paper leaves open are listed in the
 * design document and restated next to the code that implements them.
 */
#include "ig_oracle.h"

#include <algorithm>
#include <bitset>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <utility>
#include <vector>

namespace {

constexpr uint32_t NONE = IGO_NONE32;
constexpr uint16_t NONE16 = IGO_NONE16;

// ---------------------------------------------------------------------------
// Boxes: half-open integer boxes in up to three dimensions.  Unused
// dimensions are always [0,1).
// ---------------------------------------------------------------------------
struct Box {
    int64_t lo[3];
    int64_t hi[3];
};

Box make_box(const int64_t lo[3], const int64_t hi[3]) {
    Box b;
    for (int d = 0; d < 3; ++d) {
        b.lo[d] = lo[d];
        b.hi[d] = hi[d];
    }
    return b;
}

Box from_igo(const igo_box& x) { return make_box(x.min, x.max); }

igo_box to_igo(const Box& b) {
    igo_box x;
    for (int d = 0; d < 3; ++d) {
        x.min[d] = b.lo[d];
        x.max[d] = b.hi[d];
    }
    return x;
}

bool is_empty(const Box& b) {
    for (int d = 0; d < 3; ++d)
        if (b.lo[d] >= b.hi[d]) return true;
    return false;
}

Box intersect(const Box& a, const Box& b) {
    Box r;
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = std::max(a.lo[d], b.lo[d]);
        r.hi[d] = std::min(a.hi[d], b.hi[d]);
    }
    return r;
}

bool intersects(const Box& a, const Box& b) { return !is_empty(intersect(a, b)); }

// does `outer` contain every point of `inner`?
bool contains(const Box& outer, const Box& inner) {
    if (is_empty(inner)) return true;
    for (int d = 0; d < 3; ++d)
        if (inner.lo[d] < outer.lo[d] || inner.hi[d] > outer.hi[d]) return false;
    return true;
}

bool same_box(const Box& a, const Box& b) {
    for (int d = 0; d < 3; ++d)
        if (a.lo[d] != b.lo[d] || a.hi[d] != b.hi[d]) return false;
    return true;
}

bool lex_less_min(const Box& a, const Box& b) {
    for (int d = 0; d < 3; ++d)
        if (a.lo[d] != b.lo[d]) return a.lo[d] < b.lo[d];
    for (int d = 0; d < 3; ++d)
        if (a.hi[d] != b.hi[d]) return a.hi[d] < b.hi[d];
    return false;
}

Box bounding(const Box& a, const Box& b) {
    Box r;
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = std::min(a.lo[d], b.lo[d]);
        r.hi[d] = std::max(a.hi[d], b.hi[d]);
    }
    return r;
}

// a \ b as disjoint boxes: peel off the parts of `a` below and above the
// intersection, one dimension after the other.
std::vector<Box> subtract(const Box& a, const Box& b) {
    Box in = intersect(a, b);
    if (is_empty(in)) return {a};
    std::vector<Box> out;
    Box rest = a;
    for (int d = 0; d < 3; ++d) {
        if (rest.lo[d] < in.lo[d]) {
            Box p = rest;
            p.hi[d] = in.lo[d];
            out.push_back(p);
            rest.lo[d] = in.lo[d];
        }
        if (in.hi[d] < rest.hi[d]) {
            Box p = rest;
            p.lo[d] = in.hi[d];
            out.push_back(p);
            rest.hi[d] = in.hi[d];
        }
    }
    return out;
}

// A \ (union of B) for a set of disjoint boxes A.
std::vector<Box> subtract_all(std::vector<Box> a, const std::vector<Box>& bs) {
    for (const Box& b : bs) {
        std::vector<Box> next;
        for (const Box& x : a)
            for (const Box& p : subtract(x, b)) next.push_back(p);
        a.swap(next);
    }
    return a;
}

// Two boxes merge when they overlap with positive volume or share a face:
// touching in exactly one dimension while overlapping with positive length
// in the other two.  Corner or edge contact does not merge.
bool merges(const Box& a, const Box& b) {
    if (is_empty(a) || is_empty(b)) return false;
    int positive = 0, touching = 0;
    for (int d = 0; d < 3; ++d) {
        int64_t ov = std::min(a.hi[d], b.hi[d]) - std::max(a.lo[d], b.lo[d]);
        if (ov > 0)
            ++positive;
        else if (ov == 0)
            ++touching;
    }
    return positive == 3 || (positive == 2 && touching == 1);
}

// Replace merging boxes by their bounding box until no two boxes merge.
std::vector<Box> merge_fixpoint(std::vector<Box> s) {
    std::vector<Box> v;
    for (const Box& b : s)
        if (!is_empty(b)) v.push_back(b);
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t i = 0; i < v.size() && !changed; ++i)
            for (size_t j = i + 1; j < v.size() && !changed; ++j)
                if (merges(v[i], v[j])) {
                    v[i] = bounding(v[i], v[j]);
                    v.erase(v.begin() + (long)j);
                    changed = true;
                }
    }
    return v;
}

// Canonical decomposition of the union of `in` (boxes may overlap):
// dim-0-major maximal slabs.  Dimension 0 is cut only where the 2-D
// cross-section changes; inside a slab dimension 1 is cut only where the
// 1-D cross-section changes; dimension 2 uses maximal runs.  Boxes come out
// ordered by (min0, min1, min2).  The elementary grid spanned by all box
// boundaries decides membership cell by cell.
std::vector<Box> canonical(const std::vector<Box>& in) {
    std::vector<Box> boxes;
    for (const Box& b : in)
        if (!is_empty(b)) boxes.push_back(b);
    if (boxes.empty()) return {};
    std::vector<int64_t> c[3];
    for (int d = 0; d < 3; ++d) {
        for (const Box& b : boxes) {
            c[d].push_back(b.lo[d]);
            c[d].push_back(b.hi[d]);
        }
        std::sort(c[d].begin(), c[d].end());
        c[d].erase(std::unique(c[d].begin(), c[d].end()), c[d].end());
    }
    const size_t n0 = c[0].size() - 1, n1 = c[1].size() - 1, n2 = c[2].size() - 1;
    std::vector<char> cell(n0 * n1 * n2, 0);
    for (size_t i = 0; i < n0; ++i)
        for (size_t j = 0; j < n1; ++j)
            for (size_t k = 0; k < n2; ++k) {
                int64_t p[3] = {c[0][i], c[1][j], c[2][k]};
                for (const Box& b : boxes) {
                    bool inside = true;
                    for (int d = 0; d < 3; ++d)
                        if (p[d] < b.lo[d] || p[d] >= b.hi[d]) inside = false;
                    if (inside) {
                        cell[(i * n1 + j) * n2 + k] = 1;
                        break;
                    }
                }
            }
    auto at = [&](size_t i, size_t j, size_t k) { return cell[(i * n1 + j) * n2 + k] != 0; };
    auto plane_equal = [&](size_t i, size_t i2) {
        for (size_t j = 0; j < n1; ++j)
            for (size_t k = 0; k < n2; ++k)
                if (at(i, j, k) != at(i2, j, k)) return false;
        return true;
    };
    auto plane_empty = [&](size_t i) {
        for (size_t j = 0; j < n1; ++j)
            for (size_t k = 0; k < n2; ++k)
                if (at(i, j, k)) return false;
        return true;
    };
    auto line_equal = [&](size_t i, size_t j, size_t j2) {
        for (size_t k = 0; k < n2; ++k)
            if (at(i, j, k) != at(i, j2, k)) return false;
        return true;
    };
    auto line_empty = [&](size_t i, size_t j) {
        for (size_t k = 0; k < n2; ++k)
            if (at(i, j, k)) return false;
        return true;
    };
    std::vector<Box> out;
    size_t i = 0;
    while (i < n0) {
        if (plane_empty(i)) {
            ++i;
            continue;
        }
        size_t i2 = i + 1;
        while (i2 < n0 && plane_equal(i, i2)) ++i2;
        size_t j = 0;
        while (j < n1) {
            if (line_empty(i, j)) {
                ++j;
                continue;
            }
            size_t j2 = j + 1;
            while (j2 < n1 && line_equal(i, j, j2)) ++j2;
            size_t k = 0;
            while (k < n2) {
                if (!at(i, j, k)) {
                    ++k;
                    continue;
                }
                size_t k2 = k + 1;
                while (k2 < n2 && at(i, j, k2)) ++k2;
                Box b;
                b.lo[0] = c[0][i];
                b.hi[0] = c[0][i2];
                b.lo[1] = c[1][j];
                b.hi[1] = c[1][j2];
                b.lo[2] = c[2][k];
                b.hi[2] = c[2][k2];
                out.push_back(b);
                k = k2;
            }
            j = j2;
        }
        i = i2;
    }
    return out;
}

// ---------------------------------------------------------------------------
// Split and range mappers
// ---------------------------------------------------------------------------

int64_t floor_part(int64_t n, int64_t i, int64_t parts) {
    return (int64_t)(((__int128)n * i) / parts);
}

// Sec. 3.1: split dimension 0 of the task box over nodes, then the node's
// range over its devices, then the device's range into sub-chunks.
std::vector<Box> split_chunks(uint32_t nodes, uint32_t devices, uint32_t chunks, const Box& task) {
    const uint32_t per_dev = chunks / (nodes * devices);
    std::vector<Box> out(chunks);
    const int64_t lo = task.lo[0];
    const int64_t n = task.hi[0] - task.lo[0];
    for (uint32_t i = 0; i < nodes; ++i) {
        int64_t a = lo + floor_part(n, i, nodes), b = lo + floor_part(n, i + 1, nodes);
        for (uint32_t j = 0; j < devices; ++j) {
            int64_t s = a + floor_part(b - a, j, devices), e = a + floor_part(b - a, j + 1, devices);
            for (uint32_t u = 0; u < per_dev; ++u) {
                Box c = task;
                c.lo[0] = s + floor_part(e - s, u, per_dev);
                c.hi[0] = s + floor_part(e - s, u + 1, per_dev);
                out[(size_t)(i * devices + j) * per_dev + u] = c;
            }
        }
    }
    return out;
}

// Range mappers (Sec. 2.1, Listing 2): one_to_one, neighborhood, all, plus
// slice and fixed; the result is clipped to the buffer.
Box map_range(const igo_access& a, const Box& chunk, uint32_t buf_dims, const int64_t ext[3]) {
    Box r;
    for (int d = 0; d < 3; ++d) {
        r.lo[d] = 0;
        r.hi[d] = 1;
    }
    for (uint32_t d = 0; d < buf_dims; ++d) {
        switch (a.mapper) {
            case IGO_MAP_ONE_TO_ONE:
                r.lo[d] = chunk.lo[d];
                r.hi[d] = chunk.hi[d];
                break;
            case IGO_MAP_NEIGHBORHOOD:
                r.lo[d] = chunk.lo[d] - a.radius[d];
                r.hi[d] = chunk.hi[d] + a.radius[d];
                break;
            case IGO_MAP_ALL:
                r.lo[d] = 0;
                r.hi[d] = ext[d];
                break;
            case IGO_MAP_SLICE:
                if (d == a.slice_dim) {
                    r.lo[d] = 0;
                    r.hi[d] = ext[d];
                } else {
                    r.lo[d] = chunk.lo[d];
                    r.hi[d] = chunk.hi[d];
                }
                break;
            case IGO_MAP_FIXED:
                r.lo[d] = a.fixed.min[d];
                r.hi[d] = a.fixed.max[d];
                break;
        }
        r.lo[d] = std::max<int64_t>(r.lo[d], 0);
        r.hi[d] = std::min<int64_t>(r.hi[d], ext[d]);
    }
    return r;
}

// ---------------------------------------------------------------------------
// Digest: splitmix64 / FNV-1a-64 (published definitions)
// ---------------------------------------------------------------------------
uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t fnv1a64_words(const uint64_t* w, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i)
        for (int byte = 0; byte < 8; ++byte) {
            h ^= (w[i] >> (8 * byte)) & 0xFF;
            h *= 0x100000001b3ull;
        }
    return h;
}

void instruction_words(const igo_instruction& r, uint64_t w[12]) {
    w[0] = r.id;
    w[1] = (uint64_t)r.kind | ((uint64_t)r.flags << 8) | ((uint64_t)r.mem << 16) |
           ((uint64_t)r.src_mem << 32);
    w[2] = (uint64_t)r.task | ((uint64_t)r.chunk << 32);
    w[3] = r.buffer;
    w[4] = r.alloc;
    w[5] = r.src_alloc;
    for (int d = 0; d < 3; ++d) {
        w[6 + d] = (uint64_t)r.box.min[d];
        w[9 + d] = (uint64_t)r.box.max[d];
    }
}

// ---------------------------------------------------------------------------
// Context state
// ---------------------------------------------------------------------------
using MemSet = std::bitset<256>;

struct BufEntry {  // one piece of the buffer-level map
    Box box;
    uint32_t producer;  // original producer (NONE: never initialised)
    uint16_t pm;        // memory of the original producer
    MemSet mask;        // memories holding the newest data
};

struct AllocEntry {  // one piece of an allocation-level map
    Box box;
    uint32_t writer;
    std::vector<uint32_t> readers;  // sorted, unique
};

// One piece of a buffer's task-level map (Sec. 3.5 horizons from the task
// graph): the critical-path length of the element's last writer task and the
// largest one among the tasks that read it since (0 or at most the last
// epoch's: no reader).
struct CpEntry {
    Box box;
    uint32_t wcp, rcp;
};

struct Buffer {
    uint32_t dims;
    int64_t ext[3];
    uint32_t elem_size;
    uint32_t init;
    bool alive;
    uint32_t user_alloc;
    std::vector<BufEntry> map;
    std::vector<Box> initialised;  // disjoint boxes
    std::vector<CpEntry> cp_map;   // task-level map (horizon_mode 1)
    Box whole() const {
        int64_t lo[3] = {0, 0, 0};
        return make_box(lo, ext);
    }
};

struct Alloc {
    uint32_t id;
    uint16_t mem;
    uint32_t buffer;
    Box box;
    bool alive;
    std::vector<AllocEntry> map;
};

struct Region {
    uint32_t buffer;
    uint8_t mode;
    Box box;  // may be empty: no access
};

struct TaskCmd {
    uint32_t id;
    std::vector<Box> chunks;
    std::vector<std::vector<Region>> regions;  // [chunk][access]
};

struct Req {
    uint32_t buffer;
    uint16_t mem;
    Box box;
};

struct Cmd {
    bool horizon;
    TaskCmd task;
    uint32_t event;  // index of the trace event that pushed it
};

struct Access {
    uint32_t alloc;
    Box box;
    uint8_t mode;
};

struct Sources {  // incoming edges of one instruction, kinds OR-ed per source
    std::map<uint32_t, uint32_t> from;
    void add(uint32_t id, uint32_t kind) { from[id] |= kind; }
};

}  // namespace

struct igo_context {
    uint32_t nodes, devices, chunks, per_dev, horizon_step, lookahead, flush_horizons, queue_cap;
    uint32_t horizon_mode = 0, horizon_max_tasks = 0, staging = 0;
    // task graph (horizon_mode 1): critical-path lengths of the task-level
    // synchronisation point (latest epoch or applied horizon), of the latest
    // epoch, of the generated horizon not yet applied (0: none), the longest
    // path so far and its length when the last horizon or epoch came
    uint32_t cp_sync = 0, cp_epoch = 0, cp_pending = 0, cp_max = 0, cp_last = 0;
    std::vector<Buffer> buffers;
    std::vector<Alloc> allocs;  // index = allocation id; [0] unused
    std::map<std::pair<uint32_t, uint16_t>, std::vector<uint32_t>> live;
    std::vector<igo_instruction> instrs;
    std::vector<igo_binding> binds;
    std::vector<igo_edge> edges;
    std::set<uint32_t> front;
    uint32_t sync_point = 0;         // latest epoch or applied horizon
    uint32_t pending_horizon = NONE;  // emitted, not yet applied
    uint32_t tasks_since_sync = 0;
    std::deque<Cmd> queue;
    uint32_t horizons_since_alloc = 0;
    std::map<std::pair<uint32_t, uint16_t>, std::vector<Box>> plan;
    std::vector<int32_t> task_status;
    uint64_t n_tasks = 0, rejected = 0, warnings = 0, resizes = 0;
    uint64_t u_w = 0, u_r = 0, u_b = 0, map_boxes = 0;  // algorithmic-bytes terms (igo_stats)
    std::vector<igo_event> events;                      // command trace (igo_event)
    uint32_t cur_event = NONE;
    bool finished = false;
    size_t cur_instr = 0, cur_bind = 0, cur_edge = 0, cur_status = 0;

    // ----- small helpers -----
    uint32_t begin_event(uint32_t kind, uint32_t arg) {
        igo_event e;
        std::memset(&e, 0, sizeof e);
        e.kind = kind;
        e.arg = arg;
        e.compiled_at = NONE;
        e.n_instr = instrs.size();
        events.push_back(e);
        cur_event = (uint32_t)(events.size() - 1);
        return cur_event;
    }

    uint16_t mem_of_chunk(uint32_t k) const { return (uint16_t)(2 + k / per_dev); }
    uint32_t node_of_mem(uint16_t m) const { return (uint32_t)(m - 2) / devices; }

    std::vector<uint32_t>& live_list(uint32_t b, uint16_t m) { return live[{b, m}]; }

    std::vector<Box> live_boxes(uint32_t b, uint16_t m) {
        std::vector<Box> v;
        for (uint32_t a : live_list(b, m)) v.push_back(allocs[a].box);
        return v;
    }

    uint32_t alloc_containing(uint32_t b, uint16_t m, const Box& r) {
        for (uint32_t a : live_list(b, m))
            if (contains(allocs[a].box, r)) return a;
        return 0;
    }

    uint32_t emit(uint8_t kind, uint8_t flags, uint32_t task, uint32_t chunk, uint32_t buffer,
                  uint16_t mem, uint16_t src_mem, uint32_t alloc, uint32_t src_alloc, const Box& box) {
        igo_instruction r;
        std::memset(&r, 0, sizeof r);
        r.id = instrs.size();
        r.kind = kind;
        r.flags = flags;
        r.task = task;
        r.chunk = chunk;
        r.buffer = buffer;
        r.mem = mem;
        r.src_mem = src_mem;
        r.alloc = alloc;
        r.src_alloc = src_alloc;
        r.box = to_igo(box);
        instrs.push_back(r);
        return (uint32_t)r.id;
    }

    // The legend of the IDAG figure: dependencies on an allocation's creation
    // are "allocation lifetime" edges rather than data edges.
    bool is_alloc(uint32_t id) const { return instrs[id].kind == IGO_ALLOC; }

    // Close an instruction's edge list: an instruction without any data
    // dependency waits for the latest synchronisation point (the "last
    // epoch" edge kind); then the execution front moves past its sources.
    void finish(uint32_t x, Sources& s) {
        if (s.from.empty()) s.add(sync_point, IGO_DEP_SYNC);
        for (const auto& kv : s.from) {
            igo_edge e;
            std::memset(&e, 0, sizeof e);
            e.from = kv.first;
            e.to = x;
            e.kinds = kv.second;
            edges.push_back(e);
            front.erase(kv.first);
        }
        front.insert(x);
    }

    // Dataflow (true), anti and output dependencies from the allocation-level
    // maps, all evaluated against the state before instruction x.
    void access_edges(const std::vector<Access>& accs, Sources& s) {
        for (const Access& a : accs)
            for (const AllocEntry& e : allocs[a.alloc].map) {
                if (!intersects(e.box, a.box)) continue;
                if (a.mode & IGO_READ)
                    s.add(e.writer, is_alloc(e.writer) ? IGO_DEP_LIFETIME : IGO_DEP_TRUE);
                if (a.mode & IGO_WRITE) {
                    if (!e.readers.empty()) {
                        for (uint32_t r : e.readers) s.add(r, IGO_DEP_ANTI);
                    } else {
                        s.add(e.writer, is_alloc(e.writer) ? IGO_DEP_LIFETIME : IGO_DEP_OUTPUT);
                    }
                }
            }
    }

    // Record x's accesses: readers gain x, written parts get writer x and lose
    // their readers.  Reads are recorded before writes, so a part that x both
    // reads and writes ends up written.
    void access_apply(uint32_t x, const std::vector<Access>& accs) {
        for (const Access& a : accs) {
            if (a.mode & IGO_READ) ++u_r;
            if (a.mode & IGO_WRITE) ++u_w;
        }
        for (const Access& a : accs) {
            if (!(a.mode & IGO_READ)) continue;
            std::vector<AllocEntry> out;
            for (const AllocEntry& e : allocs[a.alloc].map) {
                Box in = intersect(e.box, a.box);
                if (is_empty(in)) {
                    out.push_back(e);
                    continue;
                }
                for (const Box& p : subtract(e.box, a.box)) {
                    AllocEntry c = e;
                    c.box = p;
                    out.push_back(c);
                }
                AllocEntry c = e;
                c.box = in;
                if (!std::binary_search(c.readers.begin(), c.readers.end(), x)) {
                    c.readers.push_back(x);
                    std::sort(c.readers.begin(), c.readers.end());
                }
                out.push_back(c);
            }
            allocs[a.alloc].map.swap(out);
        }
        for (const Access& a : accs) {
            if (!(a.mode & IGO_WRITE)) continue;
            std::vector<AllocEntry> out;
            for (const AllocEntry& e : allocs[a.alloc].map) {
                if (!intersects(e.box, a.box)) {
                    out.push_back(e);
                    continue;
                }
                for (const Box& p : subtract(e.box, a.box)) {
                    AllocEntry c = e;
                    c.box = p;
                    out.push_back(c);
                }
            }
            AllocEntry w;
            w.box = a.box;
            w.writer = x;
            out.push_back(w);
            allocs[a.alloc].map.swap(out);
        }
    }

    void mask_add(uint32_t b, const Box& r, uint16_t m) {
        ++u_b;
        std::vector<BufEntry> out;
        for (const BufEntry& e : buffers[b].map) {
            Box in = intersect(e.box, r);
            if (is_empty(in)) {
                out.push_back(e);
                continue;
            }
            for (const Box& p : subtract(e.box, r)) {
                BufEntry c = e;
                c.box = p;
                out.push_back(c);
            }
            BufEntry c = e;
            c.box = in;
            c.mask.set(m);
            out.push_back(c);
        }
        buffers[b].map.swap(out);
    }

    void buffer_assign(uint32_t b, const Box& r, uint32_t producer, uint16_t m) {
        ++u_b;
        std::vector<BufEntry> out;
        for (const BufEntry& e : buffers[b].map) {
            if (!intersects(e.box, r)) {
                out.push_back(e);
                continue;
            }
            for (const Box& p : subtract(e.box, r)) {
                BufEntry c = e;
                c.box = p;
                out.push_back(c);
            }
        }
        BufEntry w;
        w.box = r;
        w.producer = producer;
        w.pm = m;
        w.mask.reset();
        w.mask.set(m);
        out.push_back(w);
        buffers[b].map.swap(out);
    }

    // ----- Sec. 3.2: allocation phase of one task -----
    void allocation_phase(const TaskCmd& t, const std::vector<Req>& reqs, const std::vector<Req>& window) {
        std::set<std::pair<uint32_t, uint16_t>> pairs;  // ordered: buffer, then memory
        for (const Req& r : reqs) pairs.insert({r.buffer, r.mem});
        for (const auto& bm : pairs) {
            const uint32_t b = bm.first;
            const uint16_t m = bm.second;
            std::vector<Box> uncovered;
            for (const Req& r : reqs)
                if (r.buffer == b && r.mem == m && alloc_containing(b, m, r.box) == 0)
                    uncovered.push_back(r.box);
            if (uncovered.empty()) continue;
            std::vector<Box> pool = live_boxes(b, m);
            for (const Req& w : window)
                if (w.buffer == b && w.mem == m) pool.push_back(w.box);
            std::vector<Box> comps = merge_fixpoint(pool);
            std::vector<Box> fresh;
            for (const Box& u : uncovered)
                for (const Box& f : comps)
                    if (contains(f, u)) {
                        bool seen = false;
                        for (const Box& g : fresh) seen = seen || same_box(f, g);
                        if (!seen) fresh.push_back(f);
                        break;
                    }
            std::sort(fresh.begin(), fresh.end(), lex_less_min);
            for (const Box& nb : fresh) {
                std::vector<uint32_t> absorbed;
                for (uint32_t a : live_list(b, m))
                    if (contains(nb, allocs[a].box)) absorbed.push_back(a);
                std::sort(absorbed.begin(), absorbed.end());
                Alloc na;
                na.id = (uint32_t)allocs.size();
                na.mem = m;
                na.buffer = b;
                na.box = nb;
                na.alive = true;
                const uint32_t ai = emit(IGO_ALLOC, 0, t.id, NONE, b, m, NONE16, na.id, 0, nb);
                ++u_w;  // the new map starts with the ALLOC as writer of the whole box
                AllocEntry e0;
                e0.box = nb;
                e0.writer = ai;
                na.map.push_back(e0);
                allocs.push_back(na);
                Sources none;
                finish(ai, none);
                // resize: copy what is up to date on m out of every absorbed allocation
                for (uint32_t a : absorbed) {
                    std::vector<Box> fresh_data;
                    for (const BufEntry& e : buffers[b].map)
                        if (e.mask.test(m)) {
                            Box in = intersect(e.box, allocs[a].box);
                            if (!is_empty(in)) fresh_data.push_back(in);
                        }
                    for (const Box& cb : canonical(fresh_data)) {
                        const uint32_t ci = emit(IGO_COPY, IGO_F_RESIZE, t.id, NONE, b, m, m, na.id, a, cb);
                        std::vector<Access> acc = {{a, cb, IGO_READ}, {na.id, cb, IGO_WRITE}};
                        Sources s;
                        access_edges(acc, s);
                        finish(ci, s);
                        access_apply(ci, acc);
                    }
                }
                for (uint32_t a : absorbed) free_allocation(a, t.id);
                std::vector<uint32_t>& lst = live_list(b, m);
                std::vector<uint32_t> keep;
                for (uint32_t a : lst)
                    if (allocs[a].alive) keep.push_back(a);
                keep.push_back(na.id);
                lst.swap(keep);
                resizes += absorbed.size();
            }
        }
    }

    void free_allocation(uint32_t a, uint32_t task) {
        Alloc& al = allocs[a];
        const uint32_t fi = emit(IGO_FREE, 0, task, NONE, al.buffer, al.mem, NONE16, a, 0, al.box);
        Sources s;
        for (const AllocEntry& e : allocs[a].map) {
            s.add(e.writer, IGO_DEP_LIFETIME);
            for (uint32_t r : e.readers) s.add(r, IGO_DEP_LIFETIME);
        }
        finish(fi, s);
        allocs[a].alive = false;
    }

    // ----- Sec. 3.3: coherence copies with producer and consumer split -----
    void coherence_phase(const TaskCmd& t) {
        for (size_t k = 0; k < t.chunks.size(); ++k) {
            if (is_empty(t.chunks[k])) continue;
            const uint16_t m = mem_of_chunk((uint32_t)k);
            for (size_t j = 0; j < t.regions[k].size(); ++j) {
                const Region& rg = t.regions[k][j];
                if (!(rg.mode & IGO_READ) || is_empty(rg.box)) continue;
                const uint32_t b = rg.buffer;
                // parts of the read region that are stale on m, keyed by where
                // and by whom they were produced; uninitialised parts (no
                // memory holds them) need no copy
                std::map<std::tuple<uint16_t, uint32_t, uint32_t>, std::vector<Box>> groups;
                for (const BufEntry& e : buffers[b].map) {
                    Box need = intersect(e.box, rg.box);
                    if (is_empty(need) || e.mask.none() || e.mask.test(m)) continue;
                    // split by the source allocation on the producer's memory
                    int64_t covered = 0, total = 1;
                    for (int d = 0; d < 3; ++d) total *= need.hi[d] - need.lo[d];
                    for (uint32_t a : live_list(b, e.pm)) {
                        Box part = intersect(need, allocs[a].box);
                        if (is_empty(part)) continue;
                        int64_t v = 1;
                        for (int d = 0; d < 3; ++d) v *= part.hi[d] - part.lo[d];
                        covered += v;
                        groups[std::make_tuple(e.pm, e.producer, a)].push_back(part);
                    }
                    if (covered != total) std::abort();  // up-to-date data must be allocated
                }
                const uint32_t dst = alloc_containing(b, m, rg.box);
                if (!groups.empty() && dst == 0) std::abort();
                for (const auto& g : groups) {
                    const uint16_t src_mem = std::get<0>(g.first);
                    const uint32_t src = std::get<2>(g.first);
                    uint8_t flags = 0;
                    if (src_mem >= 2 && node_of_mem(src_mem) != node_of_mem(m)) flags |= IGO_F_INTER_NODE;
                    // without direct device-to-device copies (staging), a
                    // copy between devices of one node goes through M1
                    const bool staged = staging && src_mem >= 2 && !(flags & IGO_F_INTER_NODE);
                    for (const Box& cb : canonical(g.second)) {
                        if (staged) {
                            const uint32_t c1 = emit(IGO_COPY, 0, t.id, (uint32_t)k, b, 1, src_mem, 0, src, cb);
                            std::vector<Access> a1 = {{src, cb, IGO_READ}};
                            Sources s1;
                            access_edges(a1, s1);
                            finish(c1, s1);
                            access_apply(c1, a1);
                            const uint32_t c2 = emit(IGO_COPY, 0, t.id, (uint32_t)k, b, m, 1, dst, 0, cb);
                            std::vector<Access> a2 = {{dst, cb, IGO_WRITE}};
                            Sources s2;
                            s2.add(c1, IGO_DEP_TRUE);
                            access_edges(a2, s2);
                            finish(c2, s2);
                            access_apply(c2, a2);
                        } else {
                            const uint32_t ci = emit(IGO_COPY, flags, t.id, (uint32_t)k, b, m, src_mem, dst, src, cb);
                            std::vector<Access> acc = {{src, cb, IGO_READ}, {dst, cb, IGO_WRITE}};
                            Sources s;
                            access_edges(acc, s);
                            finish(ci, s);
                            access_apply(ci, acc);
                        }
                        mask_add(b, cb, m);
                    }
                }
            }
        }
    }

    // ----- device kernels, bindings and buffer-map update -----
    void kernel_phase(const TaskCmd& t) {
        for (size_t k = 0; k < t.chunks.size(); ++k) {
            if (is_empty(t.chunks[k])) continue;
            const uint16_t m = mem_of_chunk((uint32_t)k);
            const uint32_t ki = emit(IGO_KERNEL, 0, t.id, (uint32_t)k, NONE, m, NONE16, 0, 0, t.chunks[k]);
            std::vector<Access> acc;
            for (size_t j = 0; j < t.regions[k].size(); ++j) {
                const Region& rg = t.regions[k][j];
                uint32_t a = 0;
                if (!is_empty(rg.box)) {
                    a = alloc_containing(rg.buffer, m, rg.box);
                    if (a == 0) std::abort();
                    acc.push_back({a, rg.box, rg.mode});
                }
                igo_binding bd;
                std::memset(&bd, 0, sizeof bd);
                bd.instr = ki;
                bd.access = (uint32_t)j;
                bd.alloc = a;
                binds.push_back(bd);
            }
            Sources s;
            access_edges(acc, s);
            finish(ki, s);
            access_apply(ki, acc);
            for (size_t j = 0; j < t.regions[k].size(); ++j) {
                const Region& rg = t.regions[k][j];
                if ((rg.mode & IGO_WRITE) && !is_empty(rg.box)) buffer_assign(rg.buffer, rg.box, ki, m);
            }
        }
    }

    std::vector<Req> requirements(const TaskCmd& t) const {
        std::vector<Req> out;
        for (size_t k = 0; k < t.chunks.size(); ++k) {
            if (is_empty(t.chunks[k])) continue;
            for (const Region& rg : t.regions[k])
                if (!is_empty(rg.box)) out.push_back({rg.buffer, mem_of_chunk((uint32_t)k), rg.box});
        }
        return out;
    }

    void compile_task(const TaskCmd& t, const std::deque<Cmd>& behind) {
        std::vector<Req> reqs = requirements(t);
        std::vector<Req> window = reqs;
        for (const Cmd& c : behind)
            if (!c.horizon)
                for (const Req& r : requirements(c.task)) window.push_back(r);
        allocation_phase(t, reqs, window);
        coherence_phase(t);
        kernel_phase(t);
    }

    // Sec. 3.5: a horizon depends on the whole execution front; the previous
    // horizon becomes the new synchronisation point and replaces every older
    // producer, writer and reader in the tracking maps.
    void compile_horizon() {
        const uint32_t hi = emit(IGO_HORIZON, 0, NONE, NONE, NONE, NONE16, NONE16, 0, 0, Box{{0, 0, 0}, {0, 0, 0}});
        Sources s;
        for (uint32_t f : front) s.add(f, IGO_DEP_SYNC);
        finish(hi, s);
        if (pending_horizon != NONE) {
            const uint32_t p = pending_horizon;
            for (Buffer& bf : buffers) {
                if (!bf.alive) continue;
                for (BufEntry& e : bf.map)
                    if (e.producer != NONE && e.producer < p) e.producer = p;
            }
            for (Alloc& al : allocs) {
                if (!al.alive) continue;
                for (AllocEntry& e : al.map) {
                    if (e.writer < p) e.writer = p;
                    for (uint32_t& r : e.readers)
                        if (r < p) r = p;
                    std::sort(e.readers.begin(), e.readers.end());
                    e.readers.erase(std::unique(e.readers.begin(), e.readers.end()), e.readers.end());
                }
            }
            sync_point = p;
        }
        pending_horizon = hi;
    }

    void compile(const Cmd& c, const std::deque<Cmd>& behind) {
        events[c.event].compiled_at = cur_event;
        if (c.horizon)
            compile_horizon();
        else
            compile_task(c.task, behind);
    }

    // ----- Sec. 4.3: command queue and lookahead -----
    bool is_allocating(const TaskCmd& t) {
        for (const Req& r : requirements(t)) {
            auto it = plan.find({r.buffer, r.mem});
            std::vector<Box> v = (!queue.empty() && it != plan.end()) ? it->second : live_boxes(r.buffer, r.mem);
            bool inside = false;
            for (const Box& x : v) inside = inside || contains(x, r.box);
            if (!inside) return true;
        }
        return false;
    }

    void flush_queue() {
        while (!queue.empty()) {
            Cmd c = queue.front();
            queue.pop_front();
            compile(c, queue);
        }
        horizons_since_alloc = 0;
        plan.clear();
    }

    void push_command(const Cmd& c) {
        if (!lookahead) {
            compile(c, std::deque<Cmd>());
            return;
        }
        const bool alloc = !c.horizon && is_allocating(c.task);
        if (!c.horizon) events[c.event].allocating = alloc ? 1 : 0;
        if (queue.empty() && !alloc) {
            compile(c, std::deque<Cmd>());
            return;
        }
        queue.push_back(c);
        if (alloc) {
            horizons_since_alloc = 0;
            for (const Req& r : requirements(c.task)) {
                auto key = std::make_pair(r.buffer, r.mem);
                std::vector<Box> v = plan.count(key) ? plan[key] : live_boxes(r.buffer, r.mem);
                v.push_back(r.box);
                plan[key] = merge_fixpoint(v);
            }
        } else if (c.horizon) {
            ++horizons_since_alloc;
        }
        if (horizons_since_alloc >= flush_horizons || (queue_cap != 0 && queue.size() >= queue_cap)) flush_queue();
    }

    // ----- epoch (Sec. 2.4, Table 1) -----
    void emit_epoch() {
        flush_queue();
        const uint32_t ei = emit(IGO_EPOCH, 0, NONE, NONE, NONE, NONE16, NONE16, 0, 0, Box{{0, 0, 0}, {0, 0, 0}});
        Sources s;
        for (uint32_t f : front) s.add(f, IGO_DEP_SYNC);
        finish(ei, s);
        for (Buffer& bf : buffers) {
            if (!bf.alive) continue;
            for (BufEntry& e : bf.map)
                if (e.producer != NONE) e.producer = ei;
        }
        for (Alloc& al : allocs) {
            if (!al.alive) continue;
            for (AllocEntry& e : al.map) {
                e.writer = ei;
                e.readers.clear();
            }
        }
        sync_point = ei;
        pending_horizon = NONE;
        tasks_since_sync = 0;
        // the task graph: the epoch follows everything so far
        cp_epoch = cp_sync = cp_max = cp_last = cp_max + 1;
        cp_pending = 0;
    }

    // ----- Sec. 3.5: the task graph behind horizon_mode 1 -----
    // Critical-path length of an accepted task: one more than the longest of
    // the sync point and the tasks it depends on.  Per buffer element, over
    // the whole task's regions (every chunk; reads see the state before the
    // task): a read depends on the last writer; a write on the readers since
    // the last write, else on the last writer.  Tasks before the sync point
    // read as it (the compaction of horizons and epochs).
    uint32_t task_cp(const TaskCmd& t) {
        auto eff = [&](uint32_t v) { return v < cp_sync ? cp_sync : v; };
        uint32_t d = cp_sync;
        for (const auto& regs : t.regions)
            for (const Region& rg : regs) {
                if (is_empty(rg.box)) continue;
                for (const CpEntry& e : buffers[rg.buffer].cp_map) {
                    if (!intersects(e.box, rg.box)) continue;
                    if (rg.mode & IGO_READ) d = std::max(d, eff(e.wcp));
                    if (rg.mode & IGO_WRITE) d = std::max(d, e.rcp > cp_epoch ? eff(e.rcp) : eff(e.wcp));
                }
            }
        return d + 1;
    }

    // Record task t (critical-path length cp) in the task-level maps: reads
    // first, then writes (an element the task both reads and writes ends
    // written, with no reader).
    void task_cp_apply(const TaskCmd& t, uint32_t cp) {
        for (int pass = 0; pass < 2; ++pass)
            for (const auto& regs : t.regions)
                for (const Region& rg : regs) {
                    if (is_empty(rg.box)) continue;
                    if (pass == 0 && !(rg.mode & IGO_READ)) continue;
                    if (pass == 1 && !(rg.mode & IGO_WRITE)) continue;
                    std::vector<CpEntry> out;
                    for (const CpEntry& e : buffers[rg.buffer].cp_map) {
                        if (!intersects(e.box, rg.box)) {
                            out.push_back(e);
                            continue;
                        }
                        for (const Box& p : subtract(e.box, rg.box)) out.push_back(CpEntry{p, e.wcp, e.rcp});
                        CpEntry in{intersect(e.box, rg.box), e.wcp, e.rcp};
                        if (pass == 0) {
                            in.rcp = std::max(in.rcp > cp_epoch ? in.rcp : 0u, cp);
                        } else {
                            in.wcp = cp;
                            in.rcp = 0;
                        }
                        out.push_back(in);
                    }
                    buffers[rg.buffer].cp_map.swap(out);
                }
    }

    void destroy_buffer(uint32_t b) {
        flush_queue();
        std::vector<uint32_t> ids;
        for (auto& kv : live)
            if (kv.first.first == b && kv.first.second >= 2)
                for (uint32_t a : kv.second) ids.push_back(a);
        std::sort(ids.begin(), ids.end());
        for (uint32_t a : ids) free_allocation(a, NONE);
        for (auto& kv : live)
            if (kv.first.first == b) kv.second.clear();
        buffers[b].alive = false;
    }
};

namespace {

bool valid_box_dims(const igo_box& b, uint32_t dims) {
    for (uint32_t d = 0; d < 3; ++d) {
        if (d < dims) {
            if (b.min[d] > b.max[d]) return false;
        } else if (b.min[d] != 0 || b.max[d] != 1) {
            return false;
        }
    }
    return true;
}

template <class T>
int32_t fetch(const std::vector<T>& v, size_t& cursor, T* dst, size_t cap, size_t* n_out) {
    size_t n = std::min(cap, v.size() - cursor);
    if (n && dst) std::memcpy(dst, v.data() + cursor, n * sizeof(T));
    cursor += n;
    if (n_out) *n_out = n;
    return IGO_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int32_t igo_context_create(const igo_context_desc* d, igo_context** out) {
    if (!d || !out) return IGO_E_INVALID;
    if (d->nodes == 0 || d->devices_per_node == 0 || d->nodes * d->devices_per_node > 254) return IGO_E_INVALID;
    const uint32_t devs = d->nodes * d->devices_per_node;
    const uint32_t chunks = d->chunks ? d->chunks : devs;
    if (chunks % devs != 0 || chunks > 65536) return IGO_E_INVALID;
    if (d->lookahead > 1 || d->horizon_mode > 1) return IGO_E_INVALID;
    igo_context* c = new igo_context();
    c->nodes = d->nodes;
    c->devices = d->devices_per_node;
    c->chunks = chunks;
    c->per_dev = chunks / devs;
    c->horizon_step = d->horizon_step ? d->horizon_step : 4;
    c->lookahead = d->lookahead;
    c->flush_horizons = d->flush_horizons ? d->flush_horizons : 2;
    c->queue_cap = d->queue_cap;
    c->horizon_mode = d->horizon_mode;
    c->horizon_max_tasks = d->horizon_max_tasks ? d->horizon_max_tasks : 16 * c->horizon_step;
    c->staging = d->staging;
    c->allocs.push_back(Alloc{0, 0, 0, Box{{0, 0, 0}, {0, 0, 0}}, false, {}});
    // the initial epoch I0
    c->emit(IGO_EPOCH, 0, NONE, NONE, NONE, NONE16, NONE16, 0, 0, Box{{0, 0, 0}, {0, 0, 0}});
    c->front.insert(0);
    c->sync_point = 0;
    *out = c;
    return IGO_OK;
}

int32_t igo_context_destroy(igo_context* c) {
    if (!c) return IGO_E_INVALID;
    delete c;
    return IGO_OK;
}

int32_t igo_buffer_create(igo_context* c, uint32_t dims, const int64_t extent[3], uint32_t elem_size,
                          uint32_t init, uint32_t* out_buffer) {
    if (!c || c->finished || !extent || dims < 1 || dims > 3 || elem_size == 0 || init > 1) return IGO_E_INVALID;
    Buffer b;
    b.dims = dims;
    for (uint32_t d = 0; d < 3; ++d) {
        if (d < dims) {
            if (extent[d] < 1 || extent[d] > ((int64_t)1 << 40)) return IGO_E_INVALID;
            b.ext[d] = extent[d];
        } else {
            b.ext[d] = 1;
        }
    }
    b.elem_size = elem_size;
    b.init = init;
    b.alive = true;
    b.user_alloc = 0;
    const uint32_t id = (uint32_t)c->buffers.size();
    c->begin_event(IGO_EV_BUFFER, id);
    BufEntry e;
    e.box = b.whole();
    e.mask.reset();
    if (init == IGO_INIT_HOST) {
        // host-initialised data is up to date in user memory M0; it was
        // produced before the current synchronisation point
        Alloc ua;
        ua.id = (uint32_t)c->allocs.size();
        ua.mem = 0;
        ua.buffer = id;
        ua.box = b.whole();
        ua.alive = true;
        AllocEntry ae;
        ae.box = ua.box;
        ae.writer = c->sync_point;
        ua.map.push_back(ae);
        c->allocs.push_back(ua);
        c->live_list(id, 0).push_back(ua.id);
        b.user_alloc = ua.id;
        e.producer = c->sync_point;
        e.pm = 0;
        e.mask.set(0);
        b.initialised.push_back(b.whole());
    } else {
        e.producer = NONE;
        e.pm = NONE16;
    }
    b.map.push_back(e);
    b.cp_map.push_back(CpEntry{b.whole(), 0, 0});
    c->buffers.push_back(b);
    if (out_buffer) *out_buffer = id;
    return IGO_OK;
}

int32_t igo_buffer_destroy(igo_context* c, uint32_t b) {
    if (!c || c->finished || b >= c->buffers.size() || !c->buffers[b].alive) return IGO_E_INVALID;
    c->begin_event(IGO_EV_DESTROY, b);
    c->destroy_buffer(b);
    return IGO_OK;
}

int32_t igo_submit_task(igo_context* c, const igo_task_desc* td, uint64_t* out_task) {
    if (!c || !td || c->finished) return IGO_E_INVALID;
    if (td->dims < 1 || td->dims > 3 || td->n_access > IGO_MAX_ACCESS) return IGO_E_INVALID;
    if (!valid_box_dims(td->box, td->dims)) return IGO_E_INVALID;
    for (uint32_t j = 0; j < td->n_access; ++j) {
        const igo_access& a = td->access[j];
        if (a.buffer >= c->buffers.size() || !c->buffers[a.buffer].alive) return IGO_E_INVALID;
        if (a.mode < 1 || a.mode > 3 || a.mapper > IGO_MAP_FIXED) return IGO_E_INVALID;
        const Buffer& bf = c->buffers[a.buffer];
        const bool needs_dims = a.mapper == IGO_MAP_ONE_TO_ONE || a.mapper == IGO_MAP_NEIGHBORHOOD ||
                                a.mapper == IGO_MAP_SLICE;
        if (needs_dims && bf.dims != td->dims) return IGO_E_INVALID;
        if (a.mapper == IGO_MAP_SLICE && a.slice_dim >= bf.dims) return IGO_E_INVALID;
        if (a.mapper == IGO_MAP_NEIGHBORHOOD)
            for (uint32_t d = 0; d < bf.dims; ++d)
                if (a.radius[d] < 0) return IGO_E_INVALID;
        if (a.mapper == IGO_MAP_FIXED)
            for (uint32_t d = 0; d < bf.dims; ++d)
                if (a.fixed.min[d] > a.fixed.max[d]) return IGO_E_INVALID;
    }
    TaskCmd t;
    t.id = (uint32_t)c->n_tasks++;
    if (out_task) *out_task = t.id;
    t.chunks = split_chunks(c->nodes, c->devices, c->chunks, from_igo(td->box));
    t.regions.resize(t.chunks.size());
    for (size_t k = 0; k < t.chunks.size(); ++k) {
        for (uint32_t j = 0; j < td->n_access; ++j) {
            const igo_access& a = td->access[j];
            const Buffer& bf = c->buffers[a.buffer];
            Region rg;
            rg.buffer = a.buffer;
            rg.mode = a.mode;
            if (is_empty(t.chunks[k])) {
                rg.box = Box{{0, 0, 0}, {0, 0, 0}};
            } else {
                rg.box = map_range(a, t.chunks[k], bf.dims, bf.ext);
                if (is_empty(rg.box)) rg.box = Box{{0, 0, 0}, {0, 0, 0}};
            }
            t.regions[k].push_back(rg);
        }
        if (!is_empty(t.chunks[k])) c->map_boxes += td->n_access;
    }
    // Sec. 4.4: writes of different chunks (devices) must not overlap.  Sort
    // each buffer's write boxes by their start in dimension 0 and compare
    // every pair whose dimension-0 ranges overlap.
    std::map<uint32_t, std::vector<std::pair<Box, uint32_t>>> writes;
    for (size_t k = 0; k < t.chunks.size(); ++k)
        for (const Region& rg : t.regions[k])
            if ((rg.mode & IGO_WRITE) && !is_empty(rg.box)) writes[rg.buffer].push_back({rg.box, (uint32_t)k});
    for (auto& kv : writes) {
        auto& v = kv.second;
        std::sort(v.begin(), v.end(), [](const std::pair<Box, uint32_t>& x, const std::pair<Box, uint32_t>& y) {
            return x.first.lo[0] < y.first.lo[0];
        });
        for (size_t i = 0; i < v.size(); ++i)
            for (size_t j = i + 1; j < v.size() && v[j].first.lo[0] < v[i].first.hi[0]; ++j)
                if (v[i].second != v[j].second && intersects(v[i].first, v[j].first)) {
                    c->begin_event(IGO_EV_REJECTED, t.id);
                    c->task_status.push_back(IGO_E_OVERLAPPING_WRITE);
                    ++c->rejected;
                    return IGO_E_OVERLAPPING_WRITE;
                }
    }
    // uninitialised reads warn (the task is still accepted)
    int32_t status = IGO_OK;
    for (size_t k = 0; k < t.chunks.size(); ++k)
        for (const Region& rg : t.regions[k])
            if ((rg.mode & IGO_READ) && !is_empty(rg.box))
                if (!subtract_all({rg.box}, c->buffers[rg.buffer].initialised).empty()) status = IGO_W_UNINIT_READ;
    for (size_t k = 0; k < t.chunks.size(); ++k)
        for (const Region& rg : t.regions[k])
            if ((rg.mode & IGO_WRITE) && !is_empty(rg.box)) {
                Buffer& bf = c->buffers[rg.buffer];
                for (const Box& p : subtract_all({rg.box}, bf.initialised)) bf.initialised.push_back(p);
            }
    if (status == IGO_W_UNINIT_READ) ++c->warnings;
    c->task_status.push_back(status);
    Cmd cmd;
    cmd.horizon = false;
    cmd.task = t;
    cmd.event = c->begin_event(IGO_EV_TASK, t.id);
    c->push_command(cmd);
    // Sec. 3.5: is a horizon due after this task?
    bool horizon;
    if (c->horizon_mode == 1) {
        const uint32_t cp = c->task_cp(t);
        c->task_cp_apply(t, cp);
        c->cp_max = std::max(c->cp_max, cp);
        horizon = c->cp_max - c->cp_last >= c->horizon_step || ++c->tasks_since_sync >= c->horizon_max_tasks;
        if (horizon) {
            // the horizon follows the whole front; the one before it becomes
            // the task-level synchronisation point
            if (c->cp_pending) c->cp_sync = c->cp_pending;
            c->cp_pending = c->cp_max + 1;
            c->cp_last = c->cp_max;
        }
    } else {
        horizon = ++c->tasks_since_sync == c->horizon_step;
    }
    if (horizon) {
        c->tasks_since_sync = 0;
        Cmd h;
        h.horizon = true;
        h.event = c->begin_event(IGO_EV_HORIZON, NONE);
        c->push_command(h);
    }
    return status;
}

int32_t igo_epoch(igo_context* c) {
    if (!c || c->finished) return IGO_E_INVALID;
    c->begin_event(IGO_EV_EPOCH, NONE);
    c->emit_epoch();
    return IGO_OK;
}

int32_t igo_shutdown(igo_context* c) {
    if (!c) return IGO_E_INVALID;
    if (c->finished) return IGO_OK;
    c->begin_event(IGO_EV_SHUTDOWN, NONE);
    for (uint32_t b = 0; b < c->buffers.size(); ++b)
        if (c->buffers[b].alive) c->destroy_buffer(b);
    c->emit_epoch();
    c->finished = true;
    return IGO_OK;
}

int32_t igo_flush_window(igo_context* c) { return c ? IGO_OK : IGO_E_INVALID; }

int32_t igo_counts(igo_context* c, uint64_t* ni, uint64_t* nb, uint64_t* ne, uint64_t* nt) {
    if (!c) return IGO_E_INVALID;
    if (ni) *ni = c->instrs.size();
    if (nb) *nb = c->binds.size();
    if (ne) *ne = c->edges.size();
    if (nt) *nt = c->task_status.size();
    return IGO_OK;
}

int32_t igo_fetch_instructions(igo_context* c, igo_instruction* dst, size_t cap, size_t* n) {
    return c ? fetch(c->instrs, c->cur_instr, dst, cap, n) : IGO_E_INVALID;
}
int32_t igo_fetch_bindings(igo_context* c, igo_binding* dst, size_t cap, size_t* n) {
    return c ? fetch(c->binds, c->cur_bind, dst, cap, n) : IGO_E_INVALID;
}
int32_t igo_fetch_edges(igo_context* c, igo_edge* dst, size_t cap, size_t* n) {
    return c ? fetch(c->edges, c->cur_edge, dst, cap, n) : IGO_E_INVALID;
}
int32_t igo_fetch_task_status(igo_context* c, int32_t* dst, size_t cap, size_t* n) {
    return c ? fetch(c->task_status, c->cur_status, dst, cap, n) : IGO_E_INVALID;
}

int32_t igo_fetch_events(igo_context* c, igo_event* dst, size_t cap, size_t* n) {
    size_t cursor = 0;
    return c ? fetch(c->events, cursor, dst, cap, n) : IGO_E_INVALID;
}

size_t igo_event_count(igo_context* c) { return c ? c->events.size() : 0; }

uint64_t igo_digest(const uint64_t* words, size_t n_records, size_t wpr) {
    uint64_t sum = 0;
    for (size_t i = 0; i < n_records; ++i)
        sum += splitmix64(fnv1a64_words(words + i * wpr, wpr) ^ splitmix64((uint64_t)i));
    return sum;
}

int32_t igo_stats_get(igo_context* c, igo_stats* s) {
    if (!c || !s) return IGO_E_INVALID;
    std::memset(s, 0, sizeof *s);
    s->n_instructions = c->instrs.size();
    s->n_bindings = c->binds.size();
    s->n_edges = c->edges.size();
    for (const igo_instruction& r : c->instrs) s->per_kind[r.kind & 7]++;
    for (const igo_edge& e : c->edges)
        for (int b = 0; b < 5; ++b)
            if (e.kinds & (1u << b)) s->per_dep[b]++;
    s->resizes = c->resizes;
    s->warnings = c->warnings;
    s->tasks_submitted = c->n_tasks;
    s->tasks_rejected = c->rejected;
    s->u_w = c->u_w;
    s->u_r = c->u_r;
    s->u_b = c->u_b;
    s->map_boxes = c->map_boxes;
    uint64_t sum = 0, w[12];
    for (size_t i = 0; i < c->instrs.size(); ++i) {
        instruction_words(c->instrs[i], w);
        sum += splitmix64(fnv1a64_words(w, 12) ^ splitmix64((uint64_t)i));
    }
    s->digest_instructions = sum;
    sum = 0;
    for (size_t i = 0; i < c->binds.size(); ++i) {
        uint64_t x[3] = {c->binds[i].instr, c->binds[i].access, c->binds[i].alloc};
        sum += splitmix64(fnv1a64_words(x, 3) ^ splitmix64((uint64_t)i));
    }
    s->digest_bindings = sum;
    sum = 0;
    for (size_t i = 0; i < c->edges.size(); ++i) {
        uint64_t x[3] = {c->edges[i].from, c->edges[i].to, c->edges[i].kinds};
        sum += splitmix64(fnv1a64_words(x, 3) ^ splitmix64((uint64_t)i));
    }
    s->digest_edges = sum;
    return IGO_OK;
}

size_t igo_box_subtract(const igo_box* a, const igo_box* b, igo_box* out) {
    std::vector<Box> r = subtract(from_igo(*a), from_igo(*b));
    std::vector<Box> keep;
    for (const Box& x : r)
        if (!is_empty(x)) keep.push_back(x);
    for (size_t i = 0; i < keep.size(); ++i) out[i] = to_igo(keep[i]);
    return keep.size();
}

int32_t igo_box_merges(const igo_box* a, const igo_box* b) { return merges(from_igo(*a), from_igo(*b)) ? 1 : 0; }

size_t igo_canonical(const igo_box* in, size_t n, igo_box* out, size_t cap) {
    std::vector<Box> v;
    for (size_t i = 0; i < n; ++i) v.push_back(from_igo(in[i]));
    std::vector<Box> r = canonical(v);
    for (size_t i = 0; i < r.size() && i < cap; ++i) out[i] = to_igo(r[i]);
    return r.size();
}

size_t igo_merge_fixpoint(const igo_box* in, size_t n, igo_box* out, size_t cap) {
    std::vector<Box> v;
    for (size_t i = 0; i < n; ++i) v.push_back(from_igo(in[i]));
    std::vector<Box> r = merge_fixpoint(v);
    std::sort(r.begin(), r.end(), lex_less_min);
    for (size_t i = 0; i < r.size() && i < cap; ++i) out[i] = to_igo(r[i]);
    return r.size();
}

int32_t igo_split(uint32_t nodes, uint32_t devices, uint32_t chunks, const igo_box* task, igo_box* out) {
    if (!nodes || !devices || chunks % (nodes * devices)) return IGO_E_INVALID;
    std::vector<Box> v = split_chunks(nodes, devices, chunks, from_igo(*task));
    for (size_t i = 0; i < v.size(); ++i) out[i] = to_igo(v[i]);
    return IGO_OK;
}

int32_t igo_map(const igo_access* acc, uint32_t task_dims, const igo_box* chunk, uint32_t buf_dims,
                const int64_t extent[3], igo_box* out) {
    (void)task_dims;
    int64_t ext[3];
    for (int d = 0; d < 3; ++d) ext[d] = (uint32_t)d < buf_dims ? extent[d] : 1;
    Box r = map_range(*acc, from_igo(*chunk), buf_dims, ext);
    *out = to_igo(r);
    return IGO_OK;
}

// Sec. 4.1: the out-of-order engine, simulated (see igo_ooo_simulate in the
// header for the rules).
int32_t igo_ooo_simulate(const igo_instruction* ins, size_t n, const igo_edge* edges, size_t n_edges,
                         const igo_ooo_params* p, igo_ooo_slot* out, igo_ooo_summary* sum) {
    if ((!ins && n) || (!edges && n_edges) || !p || (!out && n) || !sum) return IGO_E_INVALID;
    if (p->lanes_per_device == 0 || p->host_lanes == 0 || p->window == 0 || p->eager > 1) return IGO_E_INVALID;
    const uint64_t INF = ~0ull;
    const uint32_t Q = p->lanes_per_device, host0 = p->devices * Q, n_lanes = host0 + p->host_lanes;
    std::vector<std::vector<uint32_t>> deps(n);
    for (size_t e = 0; e < n_edges; ++e) {
        if (edges[e].to >= n || edges[e].from >= edges[e].to) return IGO_E_INVALID;
        deps[edges[e].to].push_back((uint32_t)edges[e].from);
    }
    // the lanes an instruction may go to: [lo, hi); lo == hi: the engine's own
    std::vector<uint32_t> lo(n), hi(n);
    std::vector<uint64_t> dur(n);
    for (size_t x = 0; x < n; ++x) {
        const igo_instruction& r = ins[x];
        if (r.id != x) return IGO_E_INVALID;
        uint64_t vol = 1;
        for (int d = 0; d < 3; ++d) vol *= (uint64_t)(r.box.max[d] > r.box.min[d] ? r.box.max[d] - r.box.min[d] : 0);
        uint32_t dev = NONE;
        if (r.kind == IGO_KERNEL) {
            dev = r.mem;
            dur[x] = p->kernel_ns + vol * p->kernel_ns_per_kelem / 1024;
        } else if (r.kind == IGO_COPY) {
            dev = r.mem >= 2 ? r.mem : NONE;
            dur[x] = p->copy_ns + vol * p->copy_ns_per_kelem / 1024 + ((r.flags & IGO_F_INTER_NODE) ? p->inter_node_ns : 0);
        } else if (r.kind == IGO_ALLOC) {
            dur[x] = p->alloc_ns;
        } else if (r.kind == IGO_FREE) {
            dur[x] = p->free_ns;
        } else {
            lo[x] = hi[x] = 0;  // horizon, epoch
            dur[x] = 0;
            continue;
        }
        if (dev != NONE) {
            if (dev < 2 || dev - 2 >= p->devices) return IGO_E_INVALID;
            lo[x] = (dev - 2) * Q;
            hi[x] = lo[x] + Q;
        } else {
            lo[x] = host0;
            hi[x] = n_lanes;
        }
    }
    std::vector<bool> assigned(n, false);
    std::vector<uint64_t> end(n, INF);
    std::vector<uint64_t> busy(n_lanes, 0);
    std::memset(sum, 0, sizeof *sum);
    uint64_t t = 0;
    size_t first = 0;
    while (first < n) {
        ++sum->steps;
        while (true) {
            // which instructions are assignable at the start of this round
            const size_t last = std::min(n, first + (size_t)p->window);
            std::vector<std::pair<size_t, uint32_t>> take;  // (instruction, eager lane or NONE for direct)
            for (size_t x = first; x < last; ++x) {
                if (assigned[x]) continue;
                std::vector<uint32_t> open;
                for (uint32_t d : deps[x])
                    if (!(assigned[d] && end[d] <= t)) open.push_back(d);
                if (open.empty()) {
                    take.push_back({x, NONE});
                    continue;
                }
                if (!p->eager || lo[x] == hi[x]) continue;
                bool same = true;
                const uint32_t L = assigned[open[0]] ? out[open[0]].lane : NONE;
                for (uint32_t d : open) same = same && assigned[d] && out[d].lane == L;
                if (same && L != NONE && L >= lo[x] && L < hi[x]) take.push_back({x, L});
            }
            if (take.empty()) break;
            ++sum->rounds;
            for (const auto& tk : take) {
                const size_t x = tk.first;
                igo_ooo_slot& o = out[x];
                o.issue = t;
                if (lo[x] == hi[x]) {
                    o.lane = NONE;
                    o.how = IGO_OOO_ENGINE;
                    o.start = o.end = t;
                } else {
                    uint32_t L = tk.second;
                    if (L == NONE) {
                        L = lo[x];
                        for (uint32_t q = lo[x] + 1; q < hi[x]; ++q)
                            if (busy[q] < busy[L]) L = q;
                        o.how = IGO_OOO_DIRECT;
                        ++sum->direct;
                    } else {
                        o.how = IGO_OOO_EAGER;
                        ++sum->eager;
                    }
                    o.lane = L;
                    o.start = std::max(t, busy[L]);
                    o.end = o.start + dur[x];
                    busy[L] = o.end;
                }
                assigned[x] = true;
                end[x] = o.end;
                sum->makespan = std::max(sum->makespan, o.end);
            }
            while (first < n && assigned[first]) ++first;
        }
        if (first >= n) break;
        // the next completion
        uint64_t nt = INF;
        for (size_t x = 0; x < n; ++x)
            if (assigned[x] && end[x] > t) nt = std::min(nt, end[x]);
        if (nt == INF) return IGO_E_INVALID;  // nothing in flight and nothing assignable: not a DAG
        t = nt;
    }
    return IGO_OK;
}

}  // extern "C"
