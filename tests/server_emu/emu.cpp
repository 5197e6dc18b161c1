// CPU emulation of the device side of the serving loop (server.hip), for the
// host-logic test in tests/test_server_host_loop.py. The loop's HIP calls are
// replaced: each stream runs its queued operations in order, one at a time,
// at random moments (so completions interleave differently for each seed); a
// table copy happens when the copy runs; a batched "launch" checks, when it
// runs, that its descriptor table still holds what the host staged at launch
// time, that its (item, tile) list is a permutation of the items' tiles (a
// list split into consecutive launches is checked as a whole: every tile
// once, and the group complete by the end of the run), and that every
// element range a tile touches lies inside the operand pool and the output
// arena; at launch, no output may overlap the output of a batch the host has
// not yet seen complete.
#include <hip/hip_runtime.h>

#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "batch.hpp"
#include "salt.h"
#include "server.hpp"

static std::mt19937_64 rng(1);
static double p_step = 0.3;
static long n_errors = 0;
#define ERR(...)                         \
    do {                                 \
        if (n_errors < 30) {             \
            std::fprintf(stderr, "ERROR: "); \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fprintf(stderr, "\n");  \
        }                                \
        ++n_errors;                      \
    } while (0)

struct Range {
    uint64_t lo, hi;
};
struct PoolBuf {
    std::string name;
    uint64_t base, n, es;
};
static std::vector<PoolBuf> pools;
static uint64_t arena_lo, arena_hi;
static char *table_lo, *table_hi;

struct Op {
    int kind;  // 0 memcpy, 1 kernel, 2 event
    long seq;
    // memcpy
    char *dst = nullptr;
    const char *src = nullptr;
    size_t bytes = 0;
    // kernel
    salt::BatchLaunch L{};
    int tree = -1, dtype = -1;
    std::vector<char> expect_items, expect_tiles;
    std::vector<Range> outs;
    // event
    void *ev = nullptr;
};
struct Stream {
    std::vector<Op> q;  // pending
    long next_seq = 1, done_seq = 0;
    // the last kernel enqueued: its sequence number and item table (the
    // ranges of one split list are enqueued back to back, sharing it)
    long last_kernel_seq = -1;
    const void *last_group = nullptr;
};
struct Event {
    Stream *s = nullptr;
    long seq = 0;
    bool recorded = false;
};
static std::vector<Stream *> streams;
struct Live {
    Range r;
    Stream *s;
    long seq;  // the last launch that writes it
};
static std::vector<Live> live;  // outputs of kernels the host has not yet seen complete

static int g_tree = -1, g_dtype = -1;

// Tiles run so far of each group whose list is split over several launches,
// keyed by the group's item table; a group leaves the map when its list is
// complete.
static std::map<const void *, std::set<std::pair<int, int>>> group_seen;
static long launches = 0, split_launches = 0;

static int64_t T_of(int d) { return d == SALT_F64 ? 8192 : d == SALT_F32 ? 16384 : 32768; }
static uint64_t es_of(int d) { return d == SALT_F64 ? 8 : d == SALT_F32 ? 4 : 2; }
static int loads_of(int tree) {
    static const int L[] = {1, 1, 3, 2, 5, 3, 4, 6};  // copy scale fig1 axpy tree5 abc t4 t5
    return L[tree];
}

static void exec_kernel(Op &op) {
    const salt::BatchLaunch &L = op.L;
    const char *items_p = (const char *)L.items, *tiles_p = (const char *)L.tiles;
    if (items_p < table_lo || items_p + sizeof(salt::DevItem) * L.count > table_hi) ERR("items outside table");
    if (tiles_p < table_lo || tiles_p + sizeof(salt::TileRef) * L.total_tiles > table_hi) ERR("tiles outside table");
    if (std::memcmp(items_p, op.expect_items.data(), op.expect_items.size()))
        ERR("descriptor table changed between enqueue and execution (items)");
    if (std::memcmp(tiles_p, op.expect_tiles.data(), op.expect_tiles.size()))
        ERR("descriptor table changed between enqueue and execution (tiles)");
    const salt::DevItem *items = (const salt::DevItem *)items_p;
    const salt::TileRef *tiles = (const salt::TileRef *)tiles_p;
    const int64_t T = T_of(op.dtype);
    const uint64_t es = es_of(op.dtype);
    int64_t want_tiles = 0;
    for (int k = 0; k < L.count; ++k) want_tiles += (items[k].n + T - 1) / T;
    std::set<std::pair<int, int>> &seen = group_seen[items_p];
    ++launches;
    if (L.total_tiles != want_tiles || !seen.empty()) ++split_launches;
    for (int64_t g = 0; g < L.total_tiles; ++g) {
        const salt::TileRef r = tiles[g];
        if (r.item < 0 || r.item >= L.count) {
            ERR("bad item %d of %d", r.item, L.count);
            continue;
        }
        const salt::DevItem &it = items[r.item];
        const int64_t nt = (it.n + T - 1) / T;
        if (r.tile < 0 || r.tile >= nt) ERR("bad tile %d of %ld", r.tile, (long)nt);
        if (!seen.insert({r.item, r.tile}).second) ERR("tile listed twice");
        // address ranges one tile touches (elements [t*T, min(n, (t+1)*T)))
        const uint64_t lo = (uint64_t)r.tile * T, hi = std::min<uint64_t>(it.n, lo + T);
        const int nl = loads_of(op.tree >= 0 ? op.tree : it.tree);
        if (op.tree < 0 && (it.tree < 0 || it.tree > 7)) ERR("item names no catalogue tree");
        for (int q = 0; q < nl; ++q) {
            const uint64_t a = (uint64_t)it.ops[q] + lo * es, b = (uint64_t)it.ops[q] + hi * es;
            bool ok = false;
            for (auto &p : pools)
                if (a >= p.base && b <= p.base + p.n * p.es && p.es == es) ok = true;
            if (!ok) ERR("operand %d range outside the pool (item %d tile %d)", q, r.item, r.tile);
            if (((uint64_t)it.ops[q] & 15) && it.vec) ERR("vec set for an unaligned operand");
        }
        const uint64_t a = (uint64_t)it.out + lo * es, b = (uint64_t)it.out + hi * es;
        if (!it.out || a < arena_lo || b > arena_hi) ERR("output outside arena");
    }
    if ((int64_t)seen.size() > want_tiles) ERR("more tiles run than the group has");
    if ((int64_t)seen.size() == want_tiles) group_seen.erase(items_p);  // the group's list is complete
}

static void step(Stream *s) {
    if (s->q.empty()) return;
    Op op = s->q.front();
    s->q.erase(s->q.begin());
    if (op.kind == 0) std::memcpy(op.dst, op.src, op.bytes);
    if (op.kind == 1) exec_kernel(op);
    s->done_seq = op.seq;
}
static void maybe_progress() {
    for (auto *s : streams)
        if (std::uniform_real_distribution<double>(0, 1)(rng) < p_step) step(s);
}
static void drain(Stream *s) {
    while (!s->q.empty()) step(s);
}

extern "C" {
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    auto *st = new Stream;
    streams.push_back(st);
    *s = (hipStream_t)st;
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    Stream *st = (Stream *)s;
    for (size_t i = 0; i < streams.size(); ++i)
        if (streams[i] == st) streams.erase(streams.begin() + i);
    delete st;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) {
    for (auto *s : streams) drain(s);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    drain((Stream *)s);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) {
    *p = std::malloc(n);
    std::memset(*p, 0xcd, n);
    return hipSuccess;
}
hipError_t hipHostFree(void *p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = (hipEvent_t) new Event;
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete (Event *)e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    Event *ev = (Event *)e;
    Stream *st = (Stream *)s;
    Op op;
    op.kind = 2;
    op.seq = st->next_seq++;
    op.ev = ev;
    st->q.push_back(op);
    ev->s = st;
    ev->seq = op.seq;
    ev->recorded = true;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    Event *ev = (Event *)e;
    while (ev->s->done_seq < ev->seq) step(ev->s);
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
    Event *ev = (Event *)e;
    maybe_progress();
    if (ev->s->done_seq < ev->seq) return hipErrorNotReady;
    // the host now knows every kernel up to this event is complete
    for (size_t i = 0; i < live.size();)
        if (live[i].s == ev->s && live[i].seq <= ev->seq) live.erase(live.begin() + i);
        else ++i;
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    *ms = 0.f;
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t s) {
    Stream *st = (Stream *)s;
    if ((char *)dst < table_lo || (char *)dst + n > table_hi) ERR("memcpy destination outside the table arena");
    Op op;
    op.kind = 0;
    op.seq = st->next_seq++;
    op.dst = (char *)dst;
    op.src = (const char *)src;
    op.bytes = n;
    st->q.push_back(op);
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "emulated"; }
}

// ---- library functions the server calls --------------------------------------
namespace salt {
int64_t reduce_tile_elems(int d) { return T_of(d); }
int catalogue_loads(int id) { return loads_of(id); }
salt_status tuned_config(int, int, int, int64_t, salt_launch_config *c) {
    c->unroll = 8;
    c->nontemporal = 1;
    c->blocks = 0;
    return SALT_OK;
}
void order_tiles(TileRef *refs, int64_t count, const DevItem *items, int64_t tile_elems) {
    auto weight = [&](const TileRef &r) {
        const int64_t rest = items[r.item].n - (int64_t)r.tile * tile_elems;
        return rest < tile_elems ? rest : tile_elems;
    };
    std::stable_sort(refs, refs + count, [&](const TileRef &a, const TileRef &b) { return weight(a) > weight(b); });
}
static int stub_launch(const BatchLaunch &L) {
    Stream *st = (Stream *)L.stream;
    // a further range of the list the previous launch on this stream began
    const bool cont = st->last_group == (const void *)L.items && st->last_kernel_seq == st->next_seq - 1;
    Op op;
    op.kind = 1;
    op.seq = st->next_seq++;
    st->last_kernel_seq = op.seq;
    st->last_group = (const void *)L.items;
    op.L = L;
    op.tree = g_tree;
    op.dtype = g_dtype;
    // the bytes the kernel should see: the pending memcpy's source, now
    const char *ip = (const char *)L.items, *tp = (const char *)L.tiles;
    const Op *mc = nullptr;
    for (auto it = st->q.rbegin(); it != st->q.rend(); ++it)
        if (it->kind == 0 && ip >= it->dst && ip < it->dst + it->bytes) {
            mc = &*it;
            break;
        }
    if (!mc) {
        ERR("kernel enqueued with no pending table copy");
    } else {
        const char *src_items = mc->src + (ip - mc->dst), *src_tiles = mc->src + (tp - mc->dst);
        op.expect_items.assign(src_items, src_items + sizeof(DevItem) * L.count);
        op.expect_tiles.assign(src_tiles, src_tiles + sizeof(TileRef) * L.total_tiles);
        const DevItem *items = (const DevItem *)src_items;
        const uint64_t es = es_of(g_dtype);
        // the outputs are checked and made live by a list's first launch; its
        // further ranges write the same outputs
        if (!cont) {
            for (int k = 0; k < L.count; ++k) {
                Range r{(uint64_t)items[k].out, (uint64_t)items[k].out + (uint64_t)items[k].n * es};
                for (auto &lv : live)
                    if (r.lo < lv.r.hi && lv.r.lo < r.hi) ERR("output overlaps a live output of another batch");
                op.outs.push_back(r);
            }
            for (auto &r : op.outs) live.push_back({r, st, op.seq});
        } else {
            for (auto &lv : live)  // keep the list's outputs live until its last range completes
                if (lv.s == st && lv.seq == op.seq - 1) lv.seq = op.seq;
        }
    }
    st->q.push_back(op);
    return 0;
}
BatchFn catalogue_batch_launcher(int id, int dtype) {
    g_tree = id;
    g_dtype = dtype;
    return &stub_launch;
}
BatchFn catalogue_batch_multi_launcher(int dtype) {
    g_tree = -1;  // each item names its tree
    g_dtype = dtype;
    return &stub_launch;
}
}  // namespace salt

int main(int argc, char **argv) {
    if (argc < 9 || argc > 11) {
        std::fprintf(stderr, "usage: emu pool.txt trace.bin arena_gb p_step seed max_batch n_streams depth "
                             "[grouping [range_bytes]]\n");
        return 2;
    }
    FILE *f = std::fopen(argv[1], "r");
    if (!f) return 2;
    char name[16];
    unsigned long long base, n, es;
    while (std::fscanf(f, "%15s %llu %llu %llu", name, &base, &n, &es) == 4) pools.push_back({name, base, n, es});
    std::fclose(f);
    f = std::fopen(argv[2], "rb");
    if (!f) return 2;
    std::vector<salt_request> reqs;
    salt_request r;
    while (std::fread(&r, sizeof r, 1, f) == 1) reqs.push_back(r);
    std::fclose(f);
    const uint64_t arena_bytes = (uint64_t)std::atoll(argv[3]) << 30;
    p_step = std::atof(argv[4]);
    rng.seed(std::atoll(argv[5]));
    const int max_batch = std::atoi(argv[6]);
    const int n_streams = std::atoi(argv[7]);
    const int depth = std::atoi(argv[8]);
    arena_lo = 0x700000000000ull;
    arena_hi = arena_lo + arena_bytes;
    const size_t table_bytes = 64 << 20;
    char *table = (char *)std::aligned_alloc(256, table_bytes);
    table_lo = table;
    table_hi = table + table_bytes;
    salt_server_config cfg{};
    cfg.arena = (void *)arena_lo;
    cfg.arena_bytes = arena_bytes;
    cfg.table_arena = table;
    cfg.table_bytes = table_bytes;
    cfg.max_inflight = 4096;
    cfg.n_streams = n_streams;
    cfg.max_batch = max_batch;
    cfg.depth = depth;
    cfg.release_on_complete = 1;
    cfg.grouping = argc >= 10 ? std::atoi(argv[9]) : 0;
    cfg.range_bytes = argc >= 11 ? std::atoll(argv[10]) : 0;
    std::vector<salt_request_result> res(reqs.size());
    std::string err;
    const salt_status s = salt::serve_trace_impl(&cfg, reqs.data(), (int32_t)reqs.size(), res.data(), &err);
    int rejected = 0;
    for (auto &x : res) rejected += x.status != SALT_OK;
    if (!group_seen.empty()) ERR("%zu groups with tiles never run", group_seen.size());
    std::printf("%s: status %d (%s), %zu requests, %d rejected, %ld launches (%ld of split lists), errors %ld\n",
                argv[2], (int)s, err.c_str(), reqs.size(), rejected, launches, split_launches, n_errors);
    return n_errors ? 1 : (s != SALT_OK ? 3 : 0);
}
