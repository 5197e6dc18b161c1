// server.hip -- the serving loop (salt_serve_trace).
//
// Requests are expression evaluations over operands that stay resident in
// device memory. The loop runs on the calling thread and polls:
//   1. completions: a batched launch is done when its HIP events have fired;
//      its requests get their completion time (GPU event time mapped to the
//      host clock) and give back their slot (and their output, if asked);
//   2. arrivals: requests whose arrival time has passed join a FIFO queue;
//   3. admission: the queue head is admitted while a slot is free and its
//      output fits in the arena (first-fit allocator): memory-based
//      admission;
//   4. launch: when a stream can take another batch, every admitted request
//      not yet launched (up to max_batch) is grouped by element type; a
//      group runs as one batched launch of the mixed-tree kernel (each item
//      names its tree; batch_kernels.hpp), or is split by tree into
//      single-tree launches: always, never, or when the type's requests hold
//      many elements (the single-tree kernels stream a little faster, one
//      mixed launch finishes a small batch sooner); the groups' descriptors
//      travel in one copy from pinned staging memory.
// Requests that arrive while others run are admitted as slots and memory
// free up and overlap with them on the device (continuous batching).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "batch_ranges.hpp"
#include "expr.hpp"
#include "launch.hpp"
#include "reduce_common.hpp"
#include "server.hpp"

namespace salt {
namespace {

constexpr size_t kAlign = 256;
size_t up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
public:
    explicit Arena(size_t size) {
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = up(std::max<size_t>(bytes, 1), kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t start = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[start + bytes] = rest;
            *off = start;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = up(std::max<size_t>(bytes, 1), kAlign);
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                off = prev->first;
                bytes += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            free_.erase(next);
        }
        free_[off] = bytes;
    }

private:
    std::map<size_t, size_t> free_;
};

constexpr int kMaxGroups = 64;

struct Slot {
    int stream = 0;
    bool busy = false;
    char *dev_table = nullptr;
    char *staging = nullptr;
    size_t capacity = 0;
    std::vector<int> reqs;
    std::vector<int> group_of;  // per request in reqs: its group
    hipEvent_t ev[kMaxGroups] = {};
    int n_groups = 0;
    int batch_id = -1;
};

size_t esz(int d) { return d == SALT_F64 ? 8 : d == SALT_F32 ? 4 : 2; }

// Bytes per operand of one launch of a long group (batch_ranges.hpp). With
// several streams in flight the groups drift less than alone; measured at
// saturation (10^4 requests, three runs each): 177.3 k requests/s unsplit,
// 176.4 k at 64 MiB, 177.6 k at 128 MiB, 180.2 k at 256 MiB.
constexpr int64_t kServeRangeBytes = (int64_t)256 << 20;

}  // namespace

salt_status serve_trace_impl(const salt_server_config *cfg, const salt_request *reqs, int32_t count,
                             salt_request_result *res, std::string *err) {
    auto bad = [&](const std::string &m) {
        *err = m;
        return SALT_ERR_ARG;
    };
    if (!cfg) return bad("config is NULL");
    if (count < 0 || (count > 0 && (!reqs || !res))) return bad("bad request arrays");
    if (!cfg->arena || cfg->arena_bytes == 0) return bad("output arena missing");
    if (!cfg->table_arena || cfg->table_bytes == 0) return bad("table arena missing");
    if (cfg->max_inflight < 1 || cfg->max_batch < 1) return bad("max_inflight and max_batch must be >= 1");
    if (cfg->n_streams < 1 || cfg->n_streams > 8) return bad("n_streams outside 1..8");
    if (cfg->depth < 1 || cfg->depth > 4) return bad("depth outside 1..4");
    if (cfg->grouping < 0 || cfg->grouping > 2) return bad("grouping outside 0..2");
    if (const salt_launch_config *k = cfg->launch) {
        if (k->unroll != 0 && k->unroll != 2 && k->unroll != 4 && k->unroll != 8)
            return bad("launch unroll must be 0, 2, 4 or 8");
        if (k->nontemporal < -1 || k->nontemporal > 1) return bad("launch nontemporal outside -1..1");
        if (k->blocks < -1) return bad("launch blocks below -1");
    }
    const int n_slots = cfg->n_streams * cfg->depth;
    const size_t slot_cap = cfg->table_bytes / n_slots / kAlign * kAlign;
    if (slot_cap < 64 * 1024) return bad("table arena too small for the streams and depth");
    if (((uintptr_t)cfg->table_arena & (kAlign - 1)) || ((uintptr_t)cfg->arena & (kAlign - 1)))
        return bad("arenas must be 256-byte aligned");

    // Pre-validate every request; a bad one is rejected, the rest run.
    int n_cat = (int)cat::count;
    std::vector<char> ok(count, 1);
    for (int i = 0; i < count; ++i) {
        const salt_request &r = reqs[i];
        salt_request_result &o = res[i];
        o.arrival_s = r.arrival_s;
        o.admit_s = o.launch_s = o.complete_s = -1.0;
        o.out = nullptr;
        o.status = SALT_OK;
        o.batch = -1;
        if (i > 0 && r.arrival_s < reqs[i - 1].arrival_s) return bad("requests are not sorted by arrival time");
        int why = SALT_OK;
        if (r.tree < 0 || r.tree >= n_cat || r.dtype < SALT_F64 || r.dtype > SALT_F16 || r.n < 0)
            why = SALT_ERR_ARG;
        else if ((double)r.n * esz(r.dtype) > (double)cfg->arena_bytes)
            why = SALT_ERR_UNSUPPORTED;
        else {
            const int nl = catalogue_loads(r.tree);
            for (int k = 0; k < nl; ++k)
                if (r.n > 0 && !r.operands[k]) why = SALT_ERR_ARG;
            const int64_t T = reduce_tile_elems(r.dtype);
            const int64_t tiles = (r.n + T - 1) / T;
            if (sizeof(DevItem) + sizeof(TileRef) * (size_t)tiles + kMaxGroups * 2 * kAlign > slot_cap)
                why = SALT_ERR_UNSUPPORTED;
        }
        if (why != SALT_OK) {
            ok[i] = 0;
            o.status = why;
        }
    }

    // Streams, events, staging.
    std::vector<hipStream_t> streams(cfg->n_streams, nullptr);
    std::vector<Slot> slots(n_slots);
    hipEvent_t ev0 = nullptr;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        for (auto s : streams)
            if (s) (void)hipStreamSynchronize(s);
        for (auto &sl : slots) {
            for (auto &x : sl.ev)
                if (x) (void)hipEventDestroy(x);
            if (sl.staging) (void)hipHostFree(sl.staging);
        }
        for (auto s : streams)
            if (s) (void)hipStreamDestroy(s);
        if (ev0) (void)hipEventDestroy(ev0);
    };
    auto dev_fail = [&](hipError_t x) {
        *err = std::string("HIP error: ") + hipGetErrorString(x);
        cleanup();
        return SALT_ERR_DEVICE;
    };
    for (auto &s : streams)
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return dev_fail(e);
    for (int i = 0; i < n_slots; ++i) {
        Slot &sl = slots[i];
        sl.stream = i / cfg->depth;
        sl.capacity = slot_cap;
        sl.dev_table = (char *)cfg->table_arena + (size_t)i * slot_cap;
        if ((e = hipHostMalloc((void **)&sl.staging, slot_cap, hipHostMallocDefault)) != hipSuccess)
            return dev_fail(e);
        for (auto &x : sl.ev)
            if ((e = hipEventCreate(&x)) != hipSuccess) return dev_fail(e);
    }
    // The loop's streams do not wait for the caller's: operands (and the
    // arenas' previous users) may still be busy on other streams, so the
    // device must be idle before the first copy or launch.
    if ((e = hipDeviceSynchronize()) != hipSuccess) return dev_fail(e);
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return dev_fail(e);
    if ((e = hipEventRecord(ev0, streams[0])) != hipSuccess) return dev_fail(e);
    if ((e = hipEventSynchronize(ev0)) != hipSuccess) return dev_fail(e);
    const auto t0 = std::chrono::steady_clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };

    Arena arena(cfg->arena_bytes / kAlign * kAlign);
    std::vector<size_t> out_off(count, 0);
    std::deque<int> waiting;   // arrived, not admitted
    std::deque<int> admitted;  // admitted, not launched
    int next = 0, done = 0, inflight = 0, batches = 0;

    while (done < count) {
        bool progress = false;
        // 1. completions
        for (auto &sl : slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev[sl.n_groups - 1]);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return dev_fail(q);
            for (size_t j = 0; j < sl.reqs.size(); ++j) {
                const int r = sl.reqs[j];
                float ms = 0.f;
                if ((e = hipEventElapsedTime(&ms, ev0, sl.ev[sl.group_of[j]])) != hipSuccess) return dev_fail(e);
                res[r].complete_s = ms * 1e-3;
                if (cfg->release_on_complete) {
                    arena.release(out_off[r], (size_t)reqs[r].n * esz(reqs[r].dtype));
                    res[r].out = nullptr;
                }
                --inflight;
                ++done;
            }
            sl.busy = false;
            sl.reqs.clear();
            sl.group_of.clear();
            progress = true;
        }
        const double now = now_s();
        // 2. arrivals
        while (next < count && reqs[next].arrival_s <= now) {
            if (ok[next]) waiting.push_back(next);
            else ++done;
            ++next;
            progress = true;
        }
        // 3. admission, FIFO
        while (!waiting.empty() && inflight < cfg->max_inflight) {
            const int r = waiting.front();
            size_t off = 0;
            if (!arena.alloc((size_t)reqs[r].n * esz(reqs[r].dtype), &off)) {
                // Nothing in flight will ever return memory: with kept
                // outputs the arena is exhausted for this request.
                if (inflight == 0 && admitted.empty()) {
                    res[r].status = SALT_ERR_UNSUPPORTED;
                    waiting.pop_front();
                    ++done;
                    progress = true;
                    continue;
                }
                break;
            }
            out_off[r] = off;
            res[r].out = (char *)cfg->arena + off;
            res[r].admit_s = now;
            waiting.pop_front();
            admitted.push_back(r);
            ++inflight;
            progress = true;
        }
        // 4. launch on a stream that can take another batch
        if (!admitted.empty()) {
            Slot *free_slot = nullptr;
            for (auto &sl : slots)
                if (!sl.busy) {
                    free_slot = &sl;
                    break;
                }
            if (free_slot) {
                Slot &sl = *free_slot;
                // take requests in admission order while they fit in the table
                std::vector<int> take;
                size_t need = 0;
                while (!admitted.empty() && (int)take.size() < cfg->max_batch) {
                    const int r = admitted.front();
                    const int64_t T = reduce_tile_elems(reqs[r].dtype);
                    const size_t add = sizeof(DevItem) + sizeof(TileRef) * (size_t)((reqs[r].n + T - 1) / T);
                    if (need + add + kMaxGroups * 2 * kAlign > sl.capacity) break;
                    need += add;
                    take.push_back(r);
                    admitted.pop_front();
                }
                if (take.empty()) goto idle;
                // group by element type, and split a type's group by tree
                // as the grouping policy says; admission order is kept
                // inside a group
                int64_t type_elems[SALT_F16 + 1] = {};
                for (int r : take) type_elems[reqs[r].dtype] += reqs[r].n;
                auto split = [&](int d) {
                    return cfg->grouping == 1 || (cfg->grouping == 2 && type_elems[d] >= SALT_SERVE_SPLIT_ELEMS);
                };
                auto key = [&](int x) {
                    return std::make_pair(reqs[x].dtype, split(reqs[x].dtype) ? reqs[x].tree : -1);
                };
                std::stable_sort(take.begin(), take.end(), [&](int x, int y) { return key(x) < key(y); });
                struct Group {
                    int dtype, tree;  // tree: -1 for a mixed-tree group
                    size_t items_off, map_off;
                    int count;
                    int64_t tiles, elems;
                };
                std::vector<Group> groups;
                size_t pos = 0;
                sl.reqs.clear();
                sl.group_of.clear();
                for (size_t a = 0; a < take.size();) {
                    size_t b = a;
                    while (b < take.size() && key(take[b]) == key(take[a])) ++b;
                    Group g{reqs[take[a]].dtype, key(take[a]).second, pos, 0, (int)(b - a), 0, 0};
                    const int64_t T = reduce_tile_elems(g.dtype);
                    DevItem *items = (DevItem *)(sl.staging + pos);
                    for (size_t j = a; j < b; ++j) {
                        const salt_request &r = reqs[take[j]];
                        DevItem &d = items[j - a];
                        std::memset(&d, 0, sizeof d);
                        d.n = r.n;
                        d.tile_begin = g.tiles;
                        d.tree = r.tree;
                        bool vec = ((uintptr_t)res[take[j]].out & 15u) == 0;
                        const int nl = catalogue_loads(r.tree);
                        for (int k = 0; k < nl; ++k) {
                            d.ops[k] = r.operands[k];
                            vec = vec && (((uintptr_t)r.operands[k] & 15u) == 0);
                        }
                        for (int k = 0; k < SALT_MAX_SCALARS; ++k) {
                            d.sc64[k] = r.scalars[k];
                            d.sc32[k] = (float)r.scalars[k];
                        }
                        d.vec = vec ? 1 : 0;
                        d.out = r.n > 0 ? res[take[j]].out : nullptr;
                        g.tiles += (r.n + T - 1) / T;
                        g.elems += r.n;
                        sl.reqs.push_back(take[j]);
                        sl.group_of.push_back((int)groups.size());
                    }
                    pos = up(pos + sizeof(DevItem) * g.count, kAlign);
                    g.map_off = pos;
                    TileRef *map = (TileRef *)(sl.staging + pos);
                    int64_t t = 0;
                    for (int j = 0; j < g.count; ++j)
                        for (int64_t q = 0; q < (items[j].n + T - 1) / T; ++q) map[t++] = TileRef{j, (int32_t)q};
                    order_tiles(map, g.tiles, items, T);
                    pos = up(pos + sizeof(TileRef) * (size_t)g.tiles, kAlign);
                    groups.push_back(g);
                    a = b;
                }
                hipStream_t s = streams[sl.stream];
                if ((e = hipMemcpyAsync(sl.dev_table, sl.staging, pos, hipMemcpyHostToDevice, s)) != hipSuccess)
                    return dev_fail(e);
                for (size_t gi = 0; gi < groups.size(); ++gi) {
                    const Group &g = groups[gi];
                    // knobs of the group's tree at the size of each launch
                    // (a long tile list runs as consecutive ranges,
                    // batch_ranges.hpp); a mixed group takes those of the
                    // batched five-operand tree (the mixed-tree kernel runs
                    // 2 or 4 chunks per burst)
                    const auto knobs = [&](int64_t elems, BatchLaunch &r) -> int {
                        salt_launch_config c;
                        if (tuned_config(3, g.tree >= 0 ? g.tree : (int)cat::id_tree5, g.dtype, elems, &c) !=
                            SALT_OK) {
                            c.unroll = 4;
                            c.nontemporal = 1;
                            c.blocks = 0;
                        }
                        if (const salt_launch_config *k = cfg->launch) {  // the caller's knobs
                            if (k->unroll != 0) c.unroll = k->unroll;
                            if (k->nontemporal >= 0) c.nontemporal = k->nontemporal;
                            if (k->blocks >= 0) c.blocks = k->blocks;
                        }
                        if (g.tree < 0 && c.unroll != 2) c.unroll = 4;
                        r.unroll = c.unroll;
                        r.nontemporal = c.nontemporal;
                        r.blocks = c.blocks;
                        return 0;
                    };
                    BatchLaunch L;
                    L.items = (const DevItem *)(sl.dev_table + g.items_off);
                    L.tiles = (const TileRef *)(sl.dev_table + g.map_off);
                    L.total_tiles = g.tiles;
                    L.count = g.count;
                    L.any_dot = 0;
                    L.ws = nullptr;
                    L.stream = s;
                    L.combine = 1;
                    BatchFn fn = g.tree >= 0 ? catalogue_batch_launcher(g.tree, g.dtype)
                                             : catalogue_batch_multi_launcher(g.dtype);
                    if (!fn) return dev_fail(hipErrorInvalidValue);
                    if ((e = (hipError_t)launch_batch_ranges(fn, L, g.elems, reduce_tile_elems(g.dtype),
                                                              (int64_t)esz(g.dtype), knobs,
                                                              cfg->range_bytes ? cfg->range_bytes
                                                                               : kServeRangeBytes)) != hipSuccess)
                        return dev_fail(e);
                    if ((e = hipEventRecord(sl.ev[gi], s)) != hipSuccess) return dev_fail(e);
                }
                sl.n_groups = (int)groups.size();
                sl.busy = true;
                sl.batch_id = batches;
                for (int r : sl.reqs) {
                    res[r].launch_s = now;
                    res[r].batch = batches;
                }
                ++batches;
                progress = true;
            }
        }
    idle:
        if (!progress) std::this_thread::yield();
    }
    cleanup();
    return SALT_OK;
}

}  // namespace salt
