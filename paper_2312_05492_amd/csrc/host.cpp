// host.cpp -- the C ABI of libszi (include/szi.h): contexts, device memory
// pools, parameter checks, orchestration of the gfx950 kernels, the host
// Huffman codebook (Sec. VI-A builds it on the CPU), blob serialization.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <array>
#include <atomic>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "blob.h"
#include "szi.h"
#include "szi_internal.h"

using namespace szi;

// ------------------------------------------------------------ context
// Host worker threads that a context keeps for per-field host work of a
// batch (code books).  run(n, f) calls f(0..n-1) on the workers and the
// calling thread and returns when all calls have returned.  A worker takes
// a job's function and count under the lock and is counted busy until it
// is done with it, so run() never returns while a worker may still call f.
struct HostPool {
    std::vector<std::thread> th;
    std::mutex m;
    std::condition_variable cv, cv_done;
    const std::function<void(uint32_t)>* job = nullptr;
    uint32_t count = 0, busy = 0;
    uint64_t gen = 0;
    bool stop = false;
    std::atomic<uint32_t> next{0};

    explicit HostPool(int workers) {
        for (int t = 0; t < workers; ++t) {
            try {
                th.emplace_back([this] { work(); });
            } catch (...) {
                break;   // fewer workers; the caller does the rest
            }
        }
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(m);
            stop = true;
        }
        cv.notify_all();
        for (auto& t : th) t.join();
    }
    void work() {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(m);
        for (;;) {
            cv.wait(lk, [&] { return stop || gen != seen; });
            if (stop) return;
            seen = gen;
            const std::function<void(uint32_t)>* f = job;
            const uint32_t n = count;
            ++busy;
            lk.unlock();
            if (f)
                for (uint32_t k; (k = next.fetch_add(1)) < n;) (*f)(k);
            lk.lock();
            if (--busy == 0) cv_done.notify_all();
        }
    }
    void run(uint32_t n, const std::function<void(uint32_t)>& f) {
        {
            std::lock_guard<std::mutex> lk(m);
            job = &f;
            count = n;
            next = 0;
            ++gen;
        }
        cv.notify_all();
        for (uint32_t k; (k = next.fetch_add(1)) < n;) f(k);
        std::unique_lock<std::mutex> lk(m);
        cv_done.wait(lk, [&] { return busy == 0; });
        job = nullptr;   // a worker that wakes only now finds nothing to do
        count = 0;
    }
};

// The device bytes of a server's worker contexts together, against the
// server's budget: a worker reserves its bytes here before it allocates.
struct SharedHeld {
    std::atomic<uint64_t> held{0};
    uint64_t budget = 0;
    std::vector<sz_ctx*> ctx;
};

struct sz_ctx {
    int device = 0;
    int num_cus = 256;
    uint64_t budget = 0;       // 0 = unlimited
    uint64_t held = 0;         // bytes obtained from hipMalloc and not freed
    SharedHeld* shared = nullptr;   // a server's worker: the server's device bytes
    std::mutex pool_mu;        // pool calls may come from other threads (results freed by a server)
    std::multimap<size_t, void*> free_blocks;
    std::unordered_map<void*, size_t> block_size;
    std::string err;
    void* pinned = nullptr;    // host staging buffer
    size_t pinned_bytes = 0;
    int grid_per_cu = 0;       // persistent workgroups per CU; 0 = resident capacity
    // launch-shape tuner: the shape of each window kernel, per (kind 0 =
    // compression / 1 = replay, ndim, radius); tuned by timing the
    // candidates on the first plain call that meets a key while on
    bool tuning = false;
    std::map<std::array<int, 3>, LaunchShape> shapes;
    // graph mode: the device work of a call is captured once per launch
    // signature and replayed; its kernel arguments live in a persistent
    // device arena filled from a pinned mirror by the graph's first node
    bool graphs = false;
    hipStream_t gstream = nullptr;   // the library's stream for graph launches
    hipEvent_t gjoin = nullptr;      // joins the caller's stream to it
    void* arena = nullptr;           // device
    void* parena = nullptr;          // pinned host mirror
    size_t arena_bytes = 0;
    struct Graph {
        std::vector<uint64_t> sig;
        hipGraphExec_t exec = nullptr;
    };
    Graph graph[3];                  // decompression; compression before / after the codebook
    // stage timing
    bool timing = false;
    std::vector<hipEvent_t> ev_free;
    struct Mark {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    double stage_ms[SZ_STAGE_COUNT] = {0};
    uint64_t stage_n[SZ_STAGE_COUNT] = {0};
    std::unique_ptr<HostPool> hpool;   // made by the first batch that needs it
    void* noalloc = nullptr;           // this device's static workspace (sz_decompress_noalloc)
};

namespace {

sz_status fail(sz_ctx* c, sz_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, SZ_ERR_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                 \
    } while (0)

size_t round_block(size_t b) { return (b + 511) & ~(size_t)511; }

// Caching allocator: freed blocks are kept for reuse (every API call
// synchronizes its stream before returning, so a freed block is idle).
// a context's cached free blocks back to the device (its pool_mu held)
void drop_cache_locked(sz_ctx* c) {
    for (auto& kv : c->free_blocks) {
        (void)hipFree(kv.second);
        const size_t b = c->block_size[kv.second];
        c->held -= b;
        if (c->shared) c->shared->held -= b;
        c->block_size.erase(kv.second);
    }
    c->free_blocks.clear();
}

bool reserve_shared(SharedHeld* sh, uint64_t bytes) {
    uint64_t cur = sh->held.load();
    while (cur + bytes <= sh->budget)
        if (sh->held.compare_exchange_weak(cur, cur + bytes)) return true;
    return false;
}

sz_status pool_alloc(sz_ctx* c, size_t bytes, void** out) {
    if (bytes == 0) bytes = 1;
    bytes = round_block(bytes);
    std::unique_lock<std::mutex> lock(c->pool_mu);
    auto it = c->free_blocks.lower_bound(bytes);
    if (it != c->free_blocks.end() && it->first <= 2 * bytes + 65536) {
        *out = it->second;
        c->free_blocks.erase(it);
        return SZ_OK;
    }
    if (c->shared) {
        // a server's worker: the device bytes of all workers stay within the
        // server's budget; cached blocks go back to the device before an
        // allocation would pass it, this worker's first, then every worker's
        // (one pool lock at a time)
        SharedHeld* sh = c->shared;
        bool ok = reserve_shared(sh, bytes);
        if (!ok) {
            drop_cache_locked(c);
            ok = reserve_shared(sh, bytes);
        }
        if (!ok) {
            lock.unlock();
            for (sz_ctx* o : sh->ctx) {
                std::lock_guard<std::mutex> g(o->pool_mu);
                drop_cache_locked(o);
            }
            lock.lock();
            ok = reserve_shared(sh, bytes);
        }
        if (!ok)
            return fail(c, SZ_ERR_OOM, "server budget of %llu bytes exceeded (%llu held, %llu asked)",
                        (unsigned long long)sh->budget, (unsigned long long)sh->held.load(),
                        (unsigned long long)bytes);
    } else if (c->budget && c->held + bytes > c->budget) {
        // release cached blocks before giving up
        drop_cache_locked(c);
        if (c->held + bytes > c->budget)
            return fail(c, SZ_ERR_OOM, "device budget of %llu bytes exceeded (%llu held, %llu asked)",
                        (unsigned long long)c->budget, (unsigned long long)c->held,
                        (unsigned long long)bytes);
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        drop_cache_locked(c);
        e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (c->shared) c->shared->held -= bytes;
            return fail(c, SZ_ERR_OOM, "hipMalloc(%zu) failed", bytes);
        }
    }
    c->held += bytes;
    c->block_size[p] = bytes;
    *out = p;
    return SZ_OK;
}

void pool_free(sz_ctx* c, void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(c->pool_mu);
    auto it = c->block_size.find(p);
    if (it == c->block_size.end()) return;
    c->free_blocks.emplace(it->second, p);
}


sz_status pinned_reserve(sz_ctx* c, size_t bytes) {
    if (c->pinned_bytes >= bytes) return SZ_OK;
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_bytes = 0;
    size_t nb = std::max(bytes, (size_t)1 << 20);
    HIP_TRY(c, hipHostMalloc(&c->pinned, nb, hipHostMallocDefault));
    c->pinned_bytes = nb;
    return SZ_OK;
}

// ---- stage timing: event pairs recorded around launches, resolved after
// the call's final synchronization
hipEvent_t ev_get(sz_ctx* c) {
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

struct StageMark {
    sz_ctx* c;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr;
    StageMark(sz_ctx* cc, int s, hipStream_t stream) : c(cc), stage(s), st(stream) {
        if (c->timing && (a = ev_get(c))) (void)hipEventRecord(a, st);
    }
    ~StageMark() {
        if (!a) return;
        hipEvent_t b = ev_get(c);
        if (!b) {
            c->ev_free.push_back(a);
            return;
        }
        (void)hipEventRecord(b, st);
        c->marks.push_back({stage, a, b});
    }
};

// after the stream has synchronized
void resolve_marks(sz_ctx* c) {
    for (auto& m : c->marks) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            c->stage_ms[m.stage] += ms;
            c->stage_n[m.stage] += 1;
        } else {
            (void)hipGetLastError();
        }
        c->ev_free.push_back(m.a);
        c->ev_free.push_back(m.b);
    }
    c->marks.clear();
}

#define STAGE(c, s, st) StageMark stage_mark_##s(c, s, st)

// discards the marks of a call that ended early (declared first in a call,
// so it runs after every StageMark of that call)
struct MarkGuard {
    sz_ctx* c;
    ~MarkGuard() {
        for (auto& m : c->marks) {
            c->ev_free.push_back(m.a);
            c->ev_free.push_back(m.b);
        }
        c->marks.clear();
    }
};

// scratch allocations released together at the end of a call
struct Scratch {
    sz_ctx* c;
    std::vector<void*> blocks;
    explicit Scratch(sz_ctx* cc) : c(cc) {}
    ~Scratch() {
        for (void* p : blocks) pool_free(c, p);
    }
    template <class T>
    sz_status get(size_t count, T** out) {
        void* p;
        sz_status s = pool_alloc(c, count * sizeof(T), &p);
        if (s) return s;
        blocks.push_back(p);
        *out = static_cast<T*>(p);
        return SZ_OK;
    }
};

// ------------------------------------------------------------ graph mode
// arena layout: regions at 256-byte offsets
struct Layout {
    size_t off = 0;
    template <class T>
    size_t take(size_t count) {
        const size_t o = (off + 255) & ~(size_t)255;
        off = o + count * sizeof(T);
        return o;
    }
};

void graph_drop(sz_ctx* c) {
    for (auto& g : c->graph) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.sig.clear();
    }
}

// grow the arena (and its pinned mirror) to at least bytes; replayed graphs
// hold its addresses, so growing drops them
sz_status arena_reserve(sz_ctx* c, size_t bytes) {
    if (!c->gstream) {
        HIP_TRY(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        HIP_TRY(c, hipEventCreateWithFlags(&c->gjoin, hipEventDisableTiming));
    }
    if (bytes <= c->arena_bytes) return SZ_OK;
    HIP_TRY(c, hipStreamSynchronize(c->gstream));
    graph_drop(c);
    if (c->arena) (void)hipFree(c->arena);
    if (c->parena) (void)hipHostFree(c->parena);
    c->arena = c->parena = nullptr;
    c->arena_bytes = 0;
    const size_t nb = std::max(bytes + bytes / 2, (size_t)1 << 20);
    HIP_TRY(c, hipMalloc(&c->arena, nb));
    HIP_TRY(c, hipHostMalloc(&c->parena, nb, hipHostMallocDefault));
    c->arena_bytes = nb;
    return SZ_OK;
}

// run the launch sequence enqueue(stream) as graph g: captured on the
// library's stream when the signature is new, then replayed there after the
// caller's stream; the caller synchronizes the library's stream.  The bytes
// [soff, soff + staged) of the pinned mirror are copied to the same place in
// the arena by the graph's first node.
template <class F>
sz_status graph_run(sz_ctx* c, int g, std::vector<uint64_t> sig, size_t soff, size_t staged,
                    hipStream_t user, F&& enqueue) {
    sig.push_back(soff);
    sig.push_back(staged);
    sz_ctx::Graph& G = c->graph[g];
    HIP_TRY(c, hipEventRecord(c->gjoin, user));
    HIP_TRY(c, hipStreamWaitEvent(c->gstream, c->gjoin, 0));
    if (!G.exec || G.sig != sig) {
        if (G.exec) (void)hipGraphExecDestroy(G.exec);
        G.exec = nullptr;
        G.sig.clear();
        const bool timing = c->timing;
        c->timing = false;   // no stage events inside a graph
        HIP_TRY(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
        sz_status s = SZ_OK;
        hipError_t e = hipSuccess;
        if (staged)
            e = hipMemcpyAsync(static_cast<char*>(c->arena) + soff,
                               static_cast<char*>(c->parena) + soff, staged,
                               hipMemcpyHostToDevice, c->gstream);
        if (e == hipSuccess) s = enqueue(c->gstream);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(c->gstream, &graph);
        c->timing = timing;
        if (e != hipSuccess || e2 != hipSuccess || s != SZ_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            return s != SZ_OK ? s : fail(c, SZ_ERR_DEVICE, "graph capture failed");
        }
        const hipError_t e3 = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) {
            G.exec = nullptr;
            (void)hipGetLastError();
            return fail(c, SZ_ERR_DEVICE, "graph instantiation failed");
        }
        G.sig = sig;
    }
    HIP_TRY(c, hipGraphLaunch(G.exec, c->gstream));
    return SZ_OK;
}


// ------------------------------------------------------------ codebook
// One package-merge round: merge the sorted leaf weights lw[0, m) (lw[m] a
// sentinel) with the packages pk(j) = pw[2j] + pw[2j+1], j < np, a leaf
// first on equal weight; out[o] gets the merged weights and leaf[o] whether
// item o is a leaf.  The output is cut into four parts at their merge-path
// split points (the number of leaves among the first k items, found by
// bisection), and the four merges advance together, which gives the CPU
// four independent dependency chains instead of one.
static void merge_round(const uint64_t* lw, size_t m, const uint64_t* pw, size_t np, uint64_t* out,
                        uint8_t* leaf) {
    const size_t n = m + np;
    auto pk = [&](size_t j) { return pw[2 * j] + pw[2 * j + 1]; };
    auto corank = [&](size_t k) {
        size_t lo = k > np ? k - np : 0, hi = k < m ? k : m;
        while (lo < hi) {
            const size_t i = (lo + hi) / 2, j = k - i;
            if (j > 0 && lw[i] <= pk(j - 1)) lo = i + 1;   // leaf i precedes package j - 1
            else hi = i;
        }
        return lo;
    };
    constexpr int P = 4;
    size_t k[P + 1], i[P], j[P], ie[P], je[P];
    for (int p = 0; p <= P; ++p) k[p] = n * (size_t)p / P;
    for (int p = 0; p < P; ++p) {
        i[p] = p == 0 ? 0 : corank(k[p]);
        j[p] = k[p] - i[p];
    }
    for (int p = 0; p < P; ++p) {
        ie[p] = p + 1 < P ? i[p + 1] : m;
        je[p] = k[p + 1] - ie[p];
    }
    auto step = [&](size_t& ii, size_t& jj, size_t iie, size_t jje, size_t o) {
        const uint64_t a = lw[ii];
        const uint64_t b = jj < jje ? pk(jj) : UINT64_MAX;
        const bool tl = ii < iie && a <= b;
        out[o] = tl ? a : b;
        leaf[o] = tl;
        ii += tl;
        jj += !tl;
    };
    // each part's cursors in variables of their own, so that the four
    // chains stay in registers (indexed arrays kept them in memory: a third
    // slower)
    static_assert(P == 4, "four parts");
    size_t i0 = i[0], i1 = i[1], i2 = i[2], i3 = i[3];
    size_t j0 = j[0], j1 = j[1], j2 = j[2], j3 = j[3];
    size_t len = n;
    for (int p = 0; p < P; ++p) len = std::min(len, k[p + 1] - k[p]);
    for (size_t o = 0; o < len; ++o) {
        step(i0, j0, ie[0], je[0], k[0] + o);
        step(i1, j1, ie[1], je[1], k[1] + o);
        step(i2, j2, ie[2], je[2], k[2] + o);
        step(i3, j3, ie[3], je[3], k[3] + o);
    }
    // parts longer than the shortest
    for (size_t o = k[0] + len; o < k[1]; ++o) step(i0, j0, ie[0], je[0], o);
    for (size_t o = k[1] + len; o < k[2]; ++o) step(i1, j1, ie[1], je[1], o);
    for (size_t o = k[2] + len; o < k[3]; ++o) step(i2, j2, ie[2], je[2], o);
    for (size_t o = k[3] + len; o < k[4]; ++o) step(i3, j3, ie[3], je[3], o);
}

// Length-limited Huffman lengths by package-merge, with the tie-breaking
// fixed so that the lengths are unique: leaves ordered by (count, symbol);
// each round pairs consecutive items of the previous round's list and
// merges the pairs into the leaves, a leaf first on equal weight; the first
// 2m-2 items of the last round decide the lengths.  The leaves in a
// round's selected prefix are always the lightest ones, so a leaf's length
// is the number of rounds whose prefix holds more leaves than its rank.
void huffman_lengths(const uint32_t* h, int nsym, int lmax, uint8_t* len) {
    std::memset(len, 0, nsym);
    std::vector<uint64_t> key;   // count << 32 | symbol
    key.reserve(nsym);
    for (int s = 0; s < nsym; ++s)
        if (h[s]) key.push_back((uint64_t)h[s] << 32 | (uint32_t)s);
    const size_t m = key.size();
    if (m == 0) return;
    if (m == 1) {
        len[key[0] & 0xFFFFFFFFu] = 1;
        return;
    }
    std::sort(key.begin(), key.end());
    std::vector<uint64_t> lw(m + 1);
    for (size_t i = 0; i < m; ++i) lw[i] = key[i] >> 32;
    lw[m] = UINT64_MAX;
    const size_t cap = 2 * m;
    std::vector<uint64_t> wprev(cap), wcur(cap);
    std::vector<uint8_t> leafbit((size_t)lmax * cap);
    std::vector<size_t> lsize(lmax);
    for (size_t i = 0; i < m; ++i) {
        wprev[i] = lw[i];
        leafbit[i] = 1;
    }
    lsize[0] = m;
    for (int lv = 1; lv < lmax; ++lv) {
        const size_t np = lsize[lv - 1] / 2;
        merge_round(lw.data(), m, wprev.data(), np, wcur.data(), &leafbit[(size_t)lv * cap]);
        lsize[lv] = m + np;
        std::swap(wprev, wcur);
    }
    // rounds from the last down: the leaves among the first take items, and
    // the packages among them set the next round's take
    std::vector<int32_t> diff(m + 1, 0);
    size_t take = 2 * m - 2;
    for (int lv = lmax - 1; lv >= 0; --lv) {
        const size_t lim = std::min(take, lsize[lv]);
        const uint8_t* lb = &leafbit[(size_t)lv * cap];
        size_t nl = 0;
        for (size_t k = 0; k < lim; ++k) nl += lb[k];
        diff[0] += 1;
        diff[nl] -= 1;
        take = 2 * (lim - nl);
    }
    int32_t acc = 0;
    for (size_t i = 0; i < m; ++i) {
        acc += diff[i];
        len[key[i] & 0xFFFFFFFFu] = (uint8_t)acc;
    }
}

// canonical codewords: by length, then symbol, consecutive values
void canonical(const uint8_t* len, int nsym, uint32_t* code, uint32_t* first, uint32_t* count) {
    uint32_t nlen[kLmax + 2] = {0};
    for (int s = 0; s < nsym; ++s)
        if (len[s]) nlen[len[s]]++;
    uint32_t next[kLmax + 2] = {0};
    uint32_t c = 0;
    for (int l = 1; l <= kLmax; ++l) {
        c = (c + nlen[l - 1]) << 1;
        next[l] = c;
        if (first) first[l] = c;
        if (count) count[l] = nlen[l];
    }
    for (int s = 0; s < nsym; ++s) code[s] = len[s] ? next[len[s]]++ : 0;
}

// cbook entries (len << 24 | codeword) and the decode tables
void build_tables(const uint8_t* len, int nsym, uint32_t* cbook, uint32_t* dtab) {
    std::vector<uint32_t> code(nsym);
    uint32_t first[kLmax + 2] = {0}, count[kLmax + 2] = {0};
    canonical(len, nsym, code.data(), first, count);
    for (int s = 0; s < nsym; ++s) cbook[s] = ((uint32_t)len[s] << 24) | code[s];
    std::memset(dtab, 0, sizeof(uint32_t) * dtab_words(nsym));
    uint16_t* lut = reinterpret_cast<uint16_t*>(dtab);   // little-endian u16 view
    for (int s = 0; s < nsym; ++s) {
        const int l = len[s];
        if (l == 0 || l > kLutBits) continue;
        const uint32_t lo = code[s] << (kLutBits - l), hi = (code[s] + 1) << (kLutBits - l);
        const uint16_t e = (uint16_t)(((uint32_t)l << kLutSymBits) | (uint32_t)s);
        for (uint32_t j = lo; j < hi; ++j) lut[j] = e;
    }
    uint32_t off[kLmax + 2] = {0};   // first position of each length among the sorted symbols
    for (int l = 1; l <= kLmax; ++l) {
        off[l + 1] = off[l] + count[l];
        dtab[kDtLimit + l] = (first[l] + count[l]) << (kLmax - l);
        dtab[kDtBase + l] = off[l] - first[l];
    }
    for (int s = 0; s < nsym; ++s)
        if (len[s]) dtab[kDtSorted + off[len[s]]++] = (uint32_t)s;
}


// ------------------------------------------------------------ bookkeeping
struct ResultInternal {
    sz_ctx* owner = nullptr;       // the context whose pool holds the blocks
    std::vector<void*> blocks;     // device blocks owned by the result
    FieldPlan plan;                // host copy
    sz_dims dims;
    int S, w[3], R, chunk, eb_mode;
    double eb;
    std::vector<uint8_t> code_len; // host copy
    uint32_t* d_cbook = nullptr;
    uint32_t* d_dtab = nullptr;
    uint16_t* d_sub = nullptr;     // sub-chunk bit offsets from the encoder (null after upload)
    uint64_t nzw = UINT64_MAX;     // non-zero Huffman words; UINT64_MAX: unknown
    uint32_t* d_esec = nullptr;    // the words section with its zero words elided (device)
};

ResultInternal* ri(const sz_result* r) { return static_cast<ResultInternal*>(r->internal); }

template <class T>
sz_status res_alloc(sz_ctx* c, ResultInternal* R, size_t count, T** out) {
    void* p;
    sz_status s = pool_alloc(c, count * sizeof(T), &p);
    if (s) return s;
    R->blocks.push_back(p);
    *out = static_cast<T*>(p);
    return SZ_OK;
}

// gives one of a result's blocks back to the pool before the result is freed
void res_release(sz_ctx* c, ResultInternal* R, void* p) {
    for (size_t k = 0; k < R->blocks.size(); ++k)
        if (R->blocks[k] == p) {
            R->blocks.erase(R->blocks.begin() + k);
            pool_free(c, p);
            return;
        }
}

void release_result(sz_ctx* c, sz_result* r) {
    ResultInternal* R = ri(r);
    if (R) {
        sz_ctx* o = R->owner ? R->owner : c;
        for (void* p : R->blocks) pool_free(o, p);
        delete R;
    }
    std::memset(r, 0, sizeof(*r));
}

// the window kernels run per group of fields: 3D, 2D and 1D with the
// default stride and window, then every other geometry (the generic kernels)
constexpr int kGroups = 4, kGenGroup = 3;
inline int group_of(const Geometry& g) { return g.generic ? kGenGroup : 3 - g.ndim; }
inline int ndim_of(int group) { return 3 - group; }   // groups 0..2

hipError_t launch_compress_group(sz_ctx* c, int gi, const FieldDesc* d_fd, const FieldPlan* d_plan,
                                 const uint64_t* d_items, uint64_t nitems, LaunchShape sh, int max_R,
                                 hipStream_t q) {
    if (gi == kGenGroup) return launch_compress_gen(d_fd, d_plan, d_items, nitems, c->num_cus, max_R, q);
    return launch_compress(ndim_of(gi), d_fd, d_plan, d_items, nitems, c->num_cus, sh, max_R, q);
}

hipError_t launch_decompress_group(sz_ctx* c, int gi, const FieldDesc* d_fd, const FieldPlan* d_plan,
                                   const uint64_t* d_items, uint64_t nitems, LaunchShape sh,
                                   hipStream_t q) {
    if (gi == kGenGroup) return launch_decompress_gen(d_fd, d_plan, d_items, nitems, c->num_cus, q);
    return launch_decompress(ndim_of(gi), d_fd, d_plan, d_items, nitems, c->num_cus, sh, q);
}

// the tuner times launch shapes of the 3D and 2D default kernels only
inline bool tunable(int gi) { return gi == 0 || gi == 1; }

sz_status check_field(sz_ctx* c, const sz_dims* d, const sz_params* p, Geometry& g) {
    std::string why;
    const sz_status s = check_geometry(d, p, g, &why);
    return s ? fail(c, s, "%s", why.c_str()) : SZ_OK;
}

void fill_desc(const Geometry& g, const sz_params* p, FieldDesc& f) {
    std::memset(&f, 0, sizeof f);
    f.ndim = g.ndim;
    for (int k = 0; k < 3; ++k) {
        f.n[k] = g.n[k];
        f.w[k] = g.w[k];
        f.nwin[k] = g.nwin[k];
        f.na[k] = g.na[k];
        f.interp[k] = k < g.ndim ? p->interp[k] : 0;
        f.order_req[k] = (p->order[0] >= 0 && k < g.ndim) ? p->order[k] : -1;
    }
    f.S = g.S;
    f.L = g.L;
    f.R = g.R;
    f.chunk = g.chunk;
    f.eb_mode = p->eb_mode;
    f.eb = p->eb;
    f.alpha_req = p->alpha;
    f.npts = g.npts;
    f.nchunks = g.nchunks;
    f.need_prof = p->order[0] < 0;
    for (int k = 0; k < g.ndim; ++k)
        if (p->interp[k] == SZ_INTERP_CUBIC_AUTO) f.need_prof = 1;
}

bool words_elided(const sz_result* r, const ResultInternal* R) {
    return R->d_esec && R->nzw != UINT64_MAX && elided_words(r->n_words, R->nzw) < r->n_words;
}
uint64_t words_section_bytes(const sz_result* r, const ResultInternal* R) {
    return 4 * (words_elided(r, R) ? elided_words(r->n_words, R->nzw) : r->n_words);
}

// A result's code tables in one device block, laid out like their host
// staging: code lengths (nsym bytes, padded to 16), codebook, decode tables.
size_t tables_len_bytes(int nsym) { return ((size_t)nsym + 15) & ~(size_t)15; }
size_t tables_bytes(int nsym) {
    return tables_len_bytes(nsym) + 4 * (size_t)nsym + 4 * (size_t)dtab_words(nsym);
}

uint64_t blob_bytes(const sz_result* r, int R, uint64_t words_bytes) {
    return szi::blob_bytes(r->n_anchors, R, r->n_chunks, words_bytes, r->n_outliers);
}

// header without CRCs (they are filled by sz_serialize)
void make_header(const sz_result* r, const ResultInternal* R, uint8_t* h) {
    std::memset(h, 0, 256);
    std::memcpy(h, "SZI1", 4);
    put32(h, 4, 1);
    put32(h, 8, R->dims.ndim);
    put32(h, 12, (uint32_t)R->S);
    for (int k = 0; k < 3; ++k) {
        put64(h, 16 + 8 * k, k < (int)R->dims.ndim ? R->dims.n[k] : 0);
        put32(h, 40 + 4 * k, k < (int)R->dims.ndim ? (uint32_t)R->w[k] : 0);
    }
    put32(h, 52, (uint32_t)R->R);
    put32(h, 56, kLmax);
    put32(h, 60, (uint32_t)R->chunk);
    put32(h, 64, (uint32_t)R->eb_mode);
    put32(h, 68, (uint32_t)R->plan.levels);
    putd(h, 72, R->eb);
    putd(h, 80, R->plan.alpha);
    putf(h, 88, R->plan.vmin);
    putf(h, 92, R->plan.vmax);
    putf(h, 96, R->plan.e);
    for (int k = 0; k < 3; ++k) {
        const bool used = k < (int)R->dims.ndim;
        put32(h, 100 + 4 * k, used ? (uint32_t)R->plan.spline[k] : 0u);
        put32(h, 112 + 4 * k, used ? (uint32_t)R->plan.order[k] : 0xFFFFFFFFu);
    }
    put32(h, 124, words_elided(r, R) ? kFlagWordsElided : 0u);
    for (int l = 0; l < 16; ++l) putf(h, 128 + 4 * l, l < R->plan.levels ? R->plan.el[l] : 0.0f);
    put64(h, 192, r->n_anchors);
    put64(h, 200, r->n_chunks);
    put64(h, 208, r->n_words);
    put64(h, 216, r->n_outliers);
}

}  // namespace

// ======================================================================
// ------------------------------------------------------------ serving
// A request server: slots worker threads, each with its own context and
// stream; requests wait in arrival order and a free slot admits the oldest
// one whose device-memory estimate fits the budget that admitted requests
// and held results leave.
struct sz_server {
    int device = 0;
    uint64_t budget = 0;     // 0 = unlimited
    uint64_t charged = 0;    // estimates of running requests + bytes of held results
    std::unique_ptr<SharedHeld> shared;   // the workers' device bytes (with a budget)
    std::vector<sz_ctx*> ctx;
    std::vector<hipStream_t> st;
    std::vector<std::thread> th;
    struct Item {
        sz_request r;
        uint64_t need;
        double t_submit;
    };
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<Item> q;
    std::deque<sz_completion> done;
    std::unordered_map<void*, uint64_t> held;   // result -> bytes charged
    std::unordered_map<int32_t, std::vector<uint8_t>> books;   // resident code books
    int running = 0;
    bool stop = false;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::string err;
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Device memory a request may take while it runs: compression holds the
// codes (2 B/point), the words (at most kLmax bits per point, plus a word per
// chunk of at least 256 symbols and the slack), the elided section of the
// words while it is built (a bitmap word per 32 words, then the words), the
// outlier lists (at most 8 B per point), the call's scratch (per chunk,
// block and tile: under 1/16 B per point) and 2 MiB for per-field metadata
// and tables; the replay holds the codes.
uint64_t request_need(const sz_request& r) {
    if (r.kind == SZ_REQ_COMPRESS) {
        uint64_t n = 1;
        for (uint32_t k = 0; k < r.dims.ndim && k < 3; ++k) n *= r.dims.n[k];
        const uint64_t words = (n * kLmax + 7) / 8 + 4 * (n / 256 + 2 + kWordPad);
        return 2 * n + words + (words + words / 32 + 4) + 8 * n + n / 16 + (2u << 20);
    }
    const sz_dims& d = r.src ? ri(r.src)->dims : r.dims;
    uint64_t n = 1;
    for (uint32_t k = 0; k < d.ndim && k < 3; ++k) n *= d.n[k];
    return 2 * n + (1u << 20);
}

uint64_t result_bytes(sz_ctx* c, const sz_result* r) {
    std::lock_guard<std::mutex> lock(c->pool_mu);
    uint64_t b = 0;
    for (void* p : ri(r)->blocks) {
        auto it = c->block_size.find(p);
        if (it != c->block_size.end()) b += it->second;
    }
    return b;
}

// index of the oldest queued request that fits, or -1
long admissible(const sz_server* s) {
    for (size_t i = 0; i < s->q.size(); ++i)
        if (!s->budget || s->charged + s->q[i].need <= s->budget) return (long)i;
    return -1;
}

void server_worker(sz_server* s, int slot) {
    (void)hipSetDevice(s->device);
    sz_ctx* c = s->ctx[slot];
    for (;;) {
        std::unique_lock<std::mutex> lk(s->m);
        long pick = -1;
        s->cv_work.wait(lk, [&] {
            pick = admissible(s);
            return pick >= 0 || (s->stop && s->q.empty());
        });
        if (pick < 0) return;   // stopped and drained
        sz_server::Item it = s->q[(size_t)pick];
        s->q.erase(s->q.begin() + pick);
        s->charged += it.need;
        ++s->running;
        lk.unlock();
        sz_completion cp;
        std::memset(&cp, 0, sizeof cp);
        cp.tag = it.r.tag;
        cp.slot = slot;
        cp.t_submit = it.t_submit;
        cp.t_start = s->now();
        sz_status rc;
        // the calls return after their stream has finished the request
        if (it.r.kind == SZ_REQ_COMPRESS) {
            const uint32_t nsym = 2 * (it.r.params.radius ? it.r.params.radius : 512u);
            std::vector<uint8_t> book;
            if (it.r.book > 0) {
                std::lock_guard<std::mutex> g(s->m);
                auto b = s->books.find(it.r.book);
                if (b != s->books.end() && b->second.size() == nsym) book = b->second;
            }
            if (!book.empty()) {
                rc = sz_compress_with_code(c, it.r.d_in, &it.r.dims, &it.r.params, book.data(),
                                           s->st[slot], &cp.result);
            } else {
                rc = sz_compress(c, it.r.d_in, &it.r.dims, &it.r.params, s->st[slot], &cp.result);
                if (rc == SZ_OK && it.r.book > 0 && nsym <= 2u * kMaxRadius) {
                    // this result's histogram becomes book k
                    std::vector<uint32_t> h(nsym);
                    std::vector<uint8_t> len(nsym);
                    if (hipMemcpy(h.data(), cp.result.hist, 4 * (size_t)nsym, hipMemcpyDeviceToHost) ==
                            hipSuccess &&
                        sz_code_lengths(h.data(), nsym, len.data()) == SZ_OK) {
                        std::lock_guard<std::mutex> g(s->m);
                        auto b = s->books.find(it.r.book);
                        if (b == s->books.end() || b->second.size() != nsym) s->books[it.r.book] = len;
                    } else {
                        (void)hipGetLastError();
                    }
                }
            }
        } else {
            rc = sz_decompress(c, it.r.src, it.r.d_out, s->st[slot]);
        }
        cp.t_done = s->now();
        cp.status = rc;
        const uint64_t keep =
            (rc == SZ_OK && it.r.kind == SZ_REQ_COMPRESS) ? result_bytes(c, &cp.result) : 0;
        lk.lock();
        s->charged -= it.need;
        if (keep) {
            s->charged += keep;
            s->held[cp.result.internal] = keep;
        }
        --s->running;
        s->done.push_back(cp);
        lk.unlock();
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

}  // namespace

namespace {

// the launch shape for a window kernel: a tuned or pinned one, else the
// default; sz_ctx_set_grid overrides the grid
LaunchShape shape_for(const sz_ctx* c, int kind, int ndim, int radius) {
    auto it = c->shapes.find({kind, ndim, radius});
    LaunchShape sh = it != c->shapes.end() ? it->second : LaunchShape{};
    if (c->grid_per_cu > 0) sh.per_cu = c->grid_per_cu;
    return sh;
}

bool needs_tuning(const sz_ctx* c, int kind, int ndim, int radius) {
    return c->tuning && !c->graphs && c->grid_per_cu == 0 &&
           c->shapes.find({kind, ndim, radius}) == c->shapes.end();
}

// the candidates the tuner times: the resident grid and a smaller one; in
// 2D also the four-waves-per-SIMD variant
std::vector<LaunchShape> shape_candidates(int ndim) {
    if (ndim == 3) return {{0, 0}, {0, 2}};
    return {{0, 0}, {1, 0}, {1, 3}};
}

// Times launch(shape) for each candidate (two runs each, the faster
// counts) on stream st and returns the fastest.  The launches repeat work
// whose results the caller restores or that rewrites the same values.
template <class Launch>
sz_status tune_shapes(sz_ctx* c, int ndim, hipStream_t st, LaunchShape* best, Launch&& launch) {
    const std::vector<LaunchShape> cand = shape_candidates(ndim);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, SZ_ERR_DEVICE, "hipEventCreate");
    }
    float best_ms = 0;
    sz_status s = SZ_OK;
    for (size_t i = 0; i < cand.size() && !s; ++i) {
        float ms_min = 0;
        for (int rep = 0; rep < 2 && !s; ++rep) {
            float ms = 0;
            if (hipEventRecord(e0, st) != hipSuccess || (s = launch(cand[i])) ||
                hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                if (!s) s = fail(c, SZ_ERR_DEVICE, "timing a launch shape");
                break;
            }
            if (rep == 0 || ms < ms_min) ms_min = ms;
        }
        if (!s && (i == 0 || ms_min < best_ms)) {
            best_ms = ms_min;
            *best = cand[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}

}  // namespace

extern "C" {

sz_status sz_ctx_create(sz_ctx** out, int device, uint64_t hbm_budget_bytes) {
    if (!out) return SZ_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return SZ_ERR_DEVICE;
    }
    if (device < 0 || device >= ndev) return SZ_ERR_INVALID_ARG;
    sz_ctx* c = new sz_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return SZ_ERR_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cus = prop.multiProcessorCount;
    // the device address of the static workspace, once per device
    if (noalloc_scratch(device, &c->noalloc) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return SZ_ERR_DEVICE;
    }
    *out = c;
    return SZ_OK;
}

sz_status sz_ctx_destroy(sz_ctx* c) {
    if (!c) return SZ_OK;
    (void)hipSetDevice(c->device);
    for (auto& kv : c->block_size) {
        (void)hipFree(kv.first);
        if (c->shared) c->shared->held -= kv.second;
    }
    for (auto& m : c->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->gstream) (void)hipStreamSynchronize(c->gstream);
    graph_drop(c);
    if (c->arena) (void)hipFree(c->arena);
    if (c->parena) (void)hipHostFree(c->parena);
    if (c->gjoin) (void)hipEventDestroy(c->gjoin);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    delete c;
    return SZ_OK;
}

sz_status sz_ctx_set_graphs(sz_ctx* c, int enable) {
    if (!c) return SZ_ERR_INVALID_ARG;
    c->graphs = enable != 0;
    return SZ_OK;
}

const char* sz_last_error(const sz_ctx* c) { return c ? c->err.c_str() : "no context"; }

uint64_t sz_ctx_bytes_in_use(const sz_ctx* c) { return c ? c->held : 0; }

sz_status sz_ctx_set_timing(sz_ctx* c, int enable) {
    if (!c) return SZ_ERR_INVALID_ARG;
    c->timing = enable != 0;
    for (int k = 0; k < SZ_STAGE_COUNT; ++k) {
        c->stage_ms[k] = 0.0;
        c->stage_n[k] = 0;
    }
    return SZ_OK;
}

sz_status sz_ctx_read_timing(sz_ctx* c, double* ms, uint64_t* launches, int reset) {
    if (!c) return SZ_ERR_INVALID_ARG;
    for (int k = 0; k < SZ_STAGE_COUNT; ++k) {
        if (ms) ms[k] = c->stage_ms[k];
        if (launches) launches[k] = c->stage_n[k];
        if (reset) {
            c->stage_ms[k] = 0.0;
            c->stage_n[k] = 0;
        }
    }
    return SZ_OK;
}

// tuning hook: persistent workgroups per CU for the interpolation launches
sz_status sz_ctx_set_grid(sz_ctx* c, int workgroups_per_cu) {
    if (!c || workgroups_per_cu < 0 || workgroups_per_cu > 64) return SZ_ERR_INVALID_ARG;
    c->grid_per_cu = workgroups_per_cu;
    return SZ_OK;
}

sz_status sz_ctx_set_tuning(sz_ctx* c, int on) {
    if (!c) return SZ_ERR_INVALID_ARG;
    c->tuning = on != 0;
    return SZ_OK;
}

sz_status sz_ctx_set_shape(sz_ctx* c, int kind, int ndim, int radius, int variant,
                           int workgroups_per_cu) {
    if (!c || (kind != 0 && kind != 1) || (ndim != 2 && ndim != 3) || radius < 2 ||
        radius > kMaxRadius || variant < 0 || variant >= kShapeVariants ||
        (ndim == 3 && variant != 0) || workgroups_per_cu < 0 || workgroups_per_cu > 64)
        return SZ_ERR_INVALID_ARG;
    c->shapes[{kind, ndim, radius}] = LaunchShape{variant, workgroups_per_cu};
    return SZ_OK;
}

sz_status sz_ctx_get_shape(sz_ctx* c, int kind, int ndim, int radius, int* variant,
                           int* workgroups_per_cu, int* known) {
    if (!c || !variant || !workgroups_per_cu || !known) return SZ_ERR_INVALID_ARG;
    auto it = c->shapes.find({kind, ndim, radius});
    *known = it != c->shapes.end();
    const LaunchShape sh = *known ? it->second : LaunchShape{};
    *variant = sh.variant;
    *workgroups_per_cu = sh.per_cu;
    return SZ_OK;
}


}  // extern "C"

namespace {

// Compression of nf fields.  given: per field the caller's code lengths
// (2R entries), or null for code books built from the histograms.  With
// given code books the whole pipeline is enqueued at once and the host
// waits once, at the end, for the sizes.
sz_status compress_fields(sz_ctx* c, uint32_t nf, const float* const* d_in, const sz_dims* dims,
                          const sz_params* params, const uint8_t* const* given, void* stream,
                          sz_result* outs) {
    if (!c) return SZ_ERR_INVALID_ARG;
    if (nf == 0 || !d_in || !dims || !params || !outs)
        return fail(c, SZ_ERR_INVALID_ARG, "empty batch or null argument");
    HIP_TRY(c, hipSetDevice(c->device));
    MarkGuard mark_guard{c};
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<Geometry> geo(nf);
    std::vector<FieldDesc> fd(nf);
    for (uint32_t i = 0; i < nf; ++i) {
        if (!d_in[i]) return fail(c, SZ_ERR_INVALID_ARG, "field %u: null input", i);
        if (reinterpret_cast<uintptr_t>(d_in[i]) & 3u)
            return fail(c, SZ_ERR_INVALID_ARG, "field %u: input not 4-byte aligned", i);
        sz_status s = check_field(c, &dims[i], &params[i], geo[i]);
        if (s) return s;
        fill_desc(geo[i], &params[i], fd[i]);
        fd[i].in = d_in[i];
        if (given) {
            const uint8_t* gl = given[i];
            const int nsym = 2 * geo[i].R;
            bool ok = gl != nullptr;
            for (int sy = 0; ok && sy < nsym; ++sy) ok = gl[sy] >= 1 && gl[sy] <= kLmax;
            if (!ok || !kraft_ok(gl, nsym))
                return fail(c, SZ_ERR_INVALID_ARG,
                            "field %u: the code book must give each of the %d symbols a length "
                            "of 1..%d bits, with Kraft sum <= 1", i, nsym, kLmax);
        }
    }
    // graph mode: the launches replay from captured graphs (with a given
    // code book both graphs run back to back, without the host round trip)
    const bool graphs = c->graphs;
    // results (released on any error below)
    std::vector<sz_result> res(nf);
    std::memset(res.data(), 0, sizeof(sz_result) * nf);
    struct Guard {
        sz_ctx* c;
        std::vector<sz_result>* r;
        bool keep = false;
        ~Guard() {
            if (!keep)
                for (auto& x : *r) release_result(c, &x);
        }
    } guard{c, &res};
    uint64_t chunk_base = 0;
    int max_R = 0, max_chunk = 0;
    for (uint32_t i = 0; i < nf; ++i) {
        ResultInternal* R = new ResultInternal();
        R->owner = c;
        res[i].internal = R;
        R->dims = dims[i];
        R->S = geo[i].S;
        for (int k = 0; k < 3; ++k) R->w[k] = geo[i].w[k];
        R->R = geo[i].R;
        R->chunk = geo[i].chunk;
        R->eb_mode = params[i].eb_mode;
        R->eb = params[i].eb;
        const int nsym = 2 * geo[i].R;
        sz_status s;
        if ((s = res_alloc(c, R, geo[i].nanch, &res[i].anchors))) return s;
        if ((s = res_alloc(c, R, geo[i].npts, &res[i].codes))) return s;
        if ((s = res_alloc(c, R, nsym, &res[i].hist))) return s;
        uint8_t* tabs;   // code lengths, codebook and decode tables together
        if ((s = res_alloc(c, R, tables_bytes(nsym), &tabs))) return s;
        res[i].code_len = tabs;
        R->d_cbook = reinterpret_cast<uint32_t*>(tabs + tables_len_bytes(nsym));
        R->d_dtab = R->d_cbook + nsym;
        if ((s = res_alloc(c, R, geo[i].nchunks, &res[i].chunk_bits))) return s;
        if ((s = res_alloc(c, R, (size_t)kSubParts * geo[i].nchunks, &R->d_sub))) return s;
        res[i].n = geo[i].npts;
        res[i].n_anchors = geo[i].nanch;
        res[i].n_chunks = geo[i].nchunks;
        fd[i].codes = res[i].codes;
        fd[i].anchors = res[i].anchors;
        fd[i].hist = res[i].hist;
        fd[i].chunk_bits = res[i].chunk_bits;
        fd[i].sub = R->d_sub;
        fd[i].cbook = R->d_cbook;
        fd[i].chunk_base = chunk_base;
        chunk_base += geo[i].nchunks;
        max_R = std::max(max_R, geo[i].R);
        max_chunk = std::max(max_chunk, geo[i].chunk);
    }
    const uint64_t total_chunks = chunk_base;
    Scratch sc(c);
    sz_status s;
    // work lists: one per dimensionality, fields in input order
    std::vector<uint32_t> grp[kGroups];
    for (uint32_t i = 0; i < nf; ++i) grp[group_of(geo[i])].push_back(i);
    // stage descriptors grouped: 3D fields first, then 2D, then 1D, so that each
    // group's item offsets index a contiguous slice of the descriptor array
    std::vector<uint32_t> perm;
    for (int gi = 0; gi < kGroups; ++gi) perm.insert(perm.end(), grp[gi].begin(), grp[gi].end());
    std::vector<FieldDesc> fds(nf);
    for (uint32_t k = 0; k < nf; ++k) fds[k] = fd[perm[k]];
    std::vector<uint64_t> items(kGroups * (nf + 1), 0);
    uint64_t nitems[kGroups] = {0, 0, 0, 0};
    {
        uint32_t k = 0;
        for (int gi = 0; gi < kGroups; ++gi) {
            uint64_t* io = items.data() + gi * (nf + 1);
            io[0] = 0;
            for (size_t j = 0; j < grp[gi].size(); ++j, ++k)
                io[j + 1] = io[j] + (geo[grp[gi][j]].nwin_total + kWinPerGroup - 1) / kWinPerGroup;
            nitems[gi] = grp[gi].empty() ? 0 : io[grp[gi].size()];
        }
    }
    // Huffman encode layout.  The encode kernels are specialised on the
    // chunk size, so the fields are ordered by chunk size into contiguous
    // groups; each group runs stats -> block scan -> encode over blocks of
    // kEncBlockChunks chunks (blocks never straddle fields).
    std::vector<uint32_t> hord(nf);
    for (uint32_t k = 0; k < nf; ++k) hord[k] = k;
    std::stable_sort(hord.begin(), hord.end(),
                     [&](uint32_t x, uint32_t y) { return fds[x].chunk < fds[y].chunk; });
    std::vector<uint64_t> hboff(nf + 1, 0);   // global block prefix in hord order
    for (uint32_t j = 0; j < nf; ++j)
        hboff[j + 1] = hboff[j] + (fds[hord[j]].nchunks + kEncBlockChunks - 1) / kEncBlockChunks;
    struct Group {
        uint32_t fs, fe;   // field slice in hord order
    };
    std::vector<Group> groups;
    for (uint32_t j = 0; j < nf; ++j)
        if (groups.empty() || fds[hord[groups.back().fs]].chunk != fds[hord[j]].chunk)
            groups.push_back({j, j + 1});
        else
            groups.back().fe = j + 1;
    const uint64_t total_blocks = hboff[nf];
    // per group: block prefix (group-local) and offsets with one closing slot
    std::vector<uint64_t> gboff;            // concatenated group-local prefixes
    std::vector<uint64_t> gboff_at(groups.size()), goff_at(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        gboff_at[g] = gboff.size();
        goff_at[g] = hboff[groups[g].fs] + g;
        for (uint32_t j = groups[g].fs; j <= groups[g].fe; ++j)
            gboff.push_back(hboff[j] - hboff[groups[g].fs]);
    }
    const uint64_t nbw = total_blocks + groups.size();

    // device buffers of the launches: per-call scratch, or in graph mode the
    // arena (descriptors and offsets staged from its pinned mirror)
    FieldDesc *d_fd, *d_hfd;
    FieldPlan* d_plan;
    float *d_pmin, *d_pmax;
    uint32_t *d_pbad, *d_hist = nullptr, *d_bnz, *d_ecnt;
    unsigned long long* d_fnz;
    ElideField* d_ef;
    uint64_t *d_etoff, *d_eoff;
    char* d_scr = nullptr;   // the plain calls' scratch block
    const bool many = !graphs && nf >= 2;   // batch: gathered histograms, scattered tables
    uint64_t *d_items, *d_gboff, *d_bwoff, *d_booff;
    uint32_t *d_cwords, *d_couts, *d_bw, *d_bo;
    const size_t hstride = 2 * (size_t)max_R;   // graph mode: histogram k at d_hist + k * hstride
    Layout L;
    const size_t o_fd = L.take<FieldDesc>(nf), o_items = L.take<uint64_t>(items.size());
    const size_t end1 = L.off;
    const size_t o_plan = L.take<FieldPlan>(nf), o_hist = L.take<uint32_t>(nf * hstride);
    const size_t o_pmin = L.take<float>((size_t)nf * kRangeBlocks);
    const size_t o_pmax = L.take<float>((size_t)nf * kRangeBlocks);
    const size_t o_pbad = L.take<uint32_t>((size_t)nf * kRangeBlocks);
    const size_t o_hfd = L.take<FieldDesc>(nf), o_gboff = L.take<uint64_t>(gboff.size());
    const size_t o_ef = L.take<ElideField>(nf), o_etoff = L.take<uint64_t>(nf + 1);
    const size_t end2 = L.off;
    const size_t o_cwords = L.take<uint32_t>(std::max<uint64_t>(total_chunks, 1));
    const size_t o_couts = L.take<uint32_t>(std::max<uint64_t>(total_chunks, 1));
    const size_t o_bw = L.take<uint32_t>(std::max<uint64_t>(total_blocks, 1));
    const size_t o_bo = L.take<uint32_t>(std::max<uint64_t>(total_blocks, 1));
    const size_t o_bwoff = L.take<uint64_t>(nbw), o_booff = L.take<uint64_t>(nbw);
    const size_t o_bnz = L.take<uint32_t>(std::max<uint64_t>(total_blocks, 1));
    const size_t o_fnz = L.take<unsigned long long>(nf);
    // zero-word elision: tiles of every field's words at their largest, of
    // a size chosen from that bound
    uint64_t ewords_max = 0;
    for (uint32_t k = 0; k < nf; ++k) ewords_max += fds[k].npts * kLmax / 32 + fds[k].nchunks + 1;
    const uint64_t etw = elide_tile_words(ewords_max);
    uint64_t etiles_max = 0;
    for (uint32_t k = 0; k < nf; ++k)
        etiles_max += (fds[k].npts * kLmax / 32 + fds[k].nchunks + 1) / etw + 1;
    const size_t o_ecnt = L.take<uint32_t>(etiles_max), o_eoff = L.take<uint64_t>(etiles_max + 1);
    // host staging in pinned memory (copies from it are asynchronous): the
    // arena's layout, then each field's code lengths, codebook and decode
    // tables
    std::vector<size_t> o_cb(nf + 1);
    o_cb[0] = (L.off + 255) & ~(size_t)255;
    for (uint32_t k = 0; k < nf; ++k) {
        const size_t nsym = 2 * (size_t)fds[k].R;
        o_cb[k + 1] = o_cb[k] + ((tables_bytes((int)nsym) + 255) & ~(size_t)255);
    }
    char* hs;   // the staging base
    if (graphs) {
        if ((s = arena_reserve(c, o_cb[nf]))) return s;
        hs = static_cast<char*>(c->parena);
    } else {
        if ((s = pinned_reserve(c, o_cb[nf]))) return s;
        hs = static_cast<char*>(c->pinned);
    }
    if (graphs) {
        char* d = static_cast<char*>(c->arena);
        d_fd = reinterpret_cast<FieldDesc*>(d + o_fd);
        d_items = reinterpret_cast<uint64_t*>(d + o_items);
        d_plan = reinterpret_cast<FieldPlan*>(d + o_plan);
        d_hist = reinterpret_cast<uint32_t*>(d + o_hist);
        d_pmin = reinterpret_cast<float*>(d + o_pmin);
        d_pmax = reinterpret_cast<float*>(d + o_pmax);
        d_pbad = reinterpret_cast<uint32_t*>(d + o_pbad);
        d_hfd = reinterpret_cast<FieldDesc*>(d + o_hfd);
        d_gboff = reinterpret_cast<uint64_t*>(d + o_gboff);
        d_cwords = reinterpret_cast<uint32_t*>(d + o_cwords);
        d_couts = reinterpret_cast<uint32_t*>(d + o_couts);
        d_bw = reinterpret_cast<uint32_t*>(d + o_bw);
        d_bo = reinterpret_cast<uint32_t*>(d + o_bo);
        d_bwoff = reinterpret_cast<uint64_t*>(d + o_bwoff);
        d_booff = reinterpret_cast<uint64_t*>(d + o_booff);
        d_bnz = reinterpret_cast<uint32_t*>(d + o_bnz);
        d_ef = reinterpret_cast<ElideField*>(d + o_ef);
        d_etoff = reinterpret_cast<uint64_t*>(d + o_etoff);
        d_ecnt = reinterpret_cast<uint32_t*>(d + o_ecnt);
        d_eoff = reinterpret_cast<uint64_t*>(d + o_eoff);
        d_fnz = reinterpret_cast<unsigned long long*>(d + o_fnz);
        for (uint32_t k = 0; k < nf; ++k) fds[k].hist = d_hist + k * hstride;
    } else {
        // one scratch block in the arena's layout, so that the staged
        // regions go over in one copy each (the histograms stay in the
        // results; a batch gathers them into the block to read them back,
        // and scatters its staged code tables from the block)
        char* d;
        if ((s = sc.get(o_cb[nf], &d))) return s;
        d_scr = d;
        d_fd = reinterpret_cast<FieldDesc*>(d + o_fd);
        d_items = reinterpret_cast<uint64_t*>(d + o_items);
        d_plan = reinterpret_cast<FieldPlan*>(d + o_plan);
        d_pmin = reinterpret_cast<float*>(d + o_pmin);
        d_pmax = reinterpret_cast<float*>(d + o_pmax);
        d_pbad = reinterpret_cast<uint32_t*>(d + o_pbad);
        d_hfd = reinterpret_cast<FieldDesc*>(d + o_hfd);
        d_gboff = reinterpret_cast<uint64_t*>(d + o_gboff);
        d_cwords = reinterpret_cast<uint32_t*>(d + o_cwords);
        d_couts = reinterpret_cast<uint32_t*>(d + o_couts);
        d_bw = reinterpret_cast<uint32_t*>(d + o_bw);
        d_bo = reinterpret_cast<uint32_t*>(d + o_bo);
        d_bwoff = reinterpret_cast<uint64_t*>(d + o_bwoff);
        d_booff = reinterpret_cast<uint64_t*>(d + o_booff);
        d_bnz = reinterpret_cast<uint32_t*>(d + o_bnz);
        d_ef = reinterpret_cast<ElideField*>(d + o_ef);
        d_etoff = reinterpret_cast<uint64_t*>(d + o_etoff);
        d_ecnt = reinterpret_cast<uint32_t*>(d + o_ecnt);
        d_eoff = reinterpret_cast<uint64_t*>(d + o_eoff);
        d_fnz = reinterpret_cast<unsigned long long*>(d + o_fnz);
    }
    // the offsets and per-block counts read back at the end, one region
    const size_t o_back = o_bwoff, n_back = o_bnz + sizeof(uint32_t) * total_blocks - o_bwoff;

    // part 1: range, profile, plan (which also zeroes the histograms),
    // interpolation (with histogram)
    auto enqueue1 = [&](hipStream_t q) -> sz_status {
        {
            STAGE(c, SZ_STAGE_RANGE, q);   // with the profiling
            HIP_TRY(c, launch_range(d_fd, d_plan, (int)nf, d_pmin, d_pmax, d_pbad, q));
        }
        {
            STAGE(c, SZ_STAGE_PLAN, q);
            HIP_TRY(c, launch_plan(d_fd, d_plan, (int)nf, d_pmin, d_pmax, d_pbad, q));
        }
        uint32_t base = 0;
        for (int gi = 0; gi < kGroups; ++gi) {
            if (!grp[gi].empty()) {
                STAGE(c, SZ_STAGE_INTERP, q);
                HIP_TRY(c, launch_compress_group(c, gi, d_fd + base, d_plan + base,
                                                 d_items + gi * (nf + 1), nitems[gi],
                                                 shape_for(c, 0, ndim_of(gi), max_R), max_R, q));
            }
            base += (uint32_t)grp[gi].size();
        }
        return SZ_OK;
    };
    // plans and histograms to the staging (plain calls): a batch gathers
    // its histograms next to the plans and reads both in one copy
    auto read_plans_hists = [&](hipStream_t q) -> sz_status {
        if (many) {
            HIP_TRY(c, launch_gather_hist(d_fd, (int)nf, reinterpret_cast<uint32_t*>(d_scr + o_hist),
                                          (uint32_t)hstride, q));
            HIP_TRY(c, hipMemcpyAsync(hs + o_plan, d_plan, o_hist + sizeof(uint32_t) * nf * hstride - o_plan,
                                      hipMemcpyDeviceToHost, q));
            return SZ_OK;
        }
        HIP_TRY(c, hipMemcpyAsync(hs + o_plan, d_plan, sizeof(FieldPlan) * nf, hipMemcpyDeviceToHost, q));
        for (uint32_t k = 0; k < nf; ++k)
            HIP_TRY(c, hipMemcpyAsync(hs + o_hist + sizeof(uint32_t) * k * hstride, fds[k].hist,
                                      sizeof(uint32_t) * 2 * fds[k].R, hipMemcpyDeviceToHost, q));
        return SZ_OK;
    };
    // sync 1: plans and histograms to the host
    std::vector<FieldPlan> plans(nf);
    std::vector<std::vector<uint32_t>> hist(nf);
    for (uint32_t k = 0; k < nf; ++k) hist[k].resize(2 * fds[k].R);
    if (given && !graphs) {
        // no round trip: part 1 now, its plans and histograms read at the end
        std::memcpy(hs + o_fd, fds.data(), sizeof(FieldDesc) * nf);
        std::memcpy(hs + o_items, items.data(), sizeof(uint64_t) * items.size());
        HIP_TRY(c, hipMemcpyAsync(d_fd, hs + o_fd, end1 - o_fd, hipMemcpyHostToDevice, st));
        if ((s = enqueue1(st))) return s;
    } else if (c->graphs) {
        char* h = static_cast<char*>(c->parena);
        std::memcpy(h + o_fd, fds.data(), sizeof(FieldDesc) * nf);
        std::memcpy(h + o_items, items.data(), sizeof(uint64_t) * items.size());
        const LaunchShape s3 = shape_for(c, 0, 3, max_R), s2 = shape_for(c, 0, 2, max_R);
        const std::vector<uint64_t> sig = {nf, nitems[0], nitems[1], nitems[2], nitems[3],
                                           grp[0].size(), grp[1].size(), grp[2].size(),
                                           (uint64_t)max_R, (uint64_t)s3.per_cu, (uint64_t)s2.variant,
                                           (uint64_t)s2.per_cu, L.off};
        char* d = static_cast<char*>(c->arena);
        s = graph_run(c, 1, sig, o_fd, end1 - o_fd, st, [&](hipStream_t q) -> sz_status {
            sz_status r = enqueue1(q);
            if (r) return r;
            HIP_TRY(c, hipMemcpyAsync(h + o_plan, d + o_plan, sizeof(FieldPlan) * nf,
                                      hipMemcpyDeviceToHost, q));
            HIP_TRY(c, hipMemcpyAsync(h + o_hist, d + o_hist, sizeof(uint32_t) * nf * hstride,
                                      hipMemcpyDeviceToHost, q));
            return SZ_OK;
        });
        if (s) return s;
        if (given) {
            // no round trip: the copies of the histograms into the results
            // (on the caller's stream) wait for the graph, the plans and
            // histograms in the pinned mirror are read at the end
            HIP_TRY(c, hipEventRecord(c->gjoin, c->gstream));
            HIP_TRY(c, hipStreamWaitEvent(st, c->gjoin, 0));
        } else {
            HIP_TRY(c, hipStreamSynchronize(c->gstream));
            std::memcpy(plans.data(), h + o_plan, sizeof(FieldPlan) * nf);
            for (uint32_t k = 0; k < nf; ++k)
                std::memcpy(hist[k].data(), h + o_hist + sizeof(uint32_t) * k * hstride,
                            sizeof(uint32_t) * hist[k].size());
        }
    } else {
        std::memcpy(hs + o_fd, fds.data(), sizeof(FieldDesc) * nf);
        std::memcpy(hs + o_items, items.data(), sizeof(uint64_t) * items.size());
        HIP_TRY(c, hipMemcpyAsync(d_fd, hs + o_fd, end1 - o_fd, hipMemcpyHostToDevice, st));
        if ((s = enqueue1(st))) return s;
        if ((s = read_plans_hists(st))) return s;
        HIP_TRY(c, hipStreamSynchronize(st));
        std::memcpy(plans.data(), hs + o_plan, sizeof(FieldPlan) * nf);
        for (uint32_t k = 0; k < nf; ++k)
            std::memcpy(hist[k].data(), hs + o_hist + sizeof(uint32_t) * k * hstride,
                        sizeof(uint32_t) * hist[k].size());
        // launch-shape tuning: the interpolation launch of a group again per
        // candidate (same codes and anchors; the histograms gain counts),
        // then the histograms rebuilt with the chosen shapes
        bool tuned = false;
        uint32_t base = 0;
        for (int gi = 0; gi < kGroups; ++gi) {
            const int nd = ndim_of(gi);
            if (!grp[gi].empty() && tunable(gi) && needs_tuning(c, 0, nd, max_R)) {
                LaunchShape best;
                s = tune_shapes(c, nd, st, &best, [&](LaunchShape sh) -> sz_status {
                    HIP_TRY(c, launch_compress(nd, d_fd + base, d_plan + base, d_items + gi * (nf + 1),
                                               nitems[gi], c->num_cus, sh, max_R, st));
                    return SZ_OK;
                });
                if (s) return s;
                c->shapes[{0, nd, max_R}] = best;
                tuned = true;
            }
            base += (uint32_t)grp[gi].size();
        }
        if (tuned) {
            HIP_TRY(c, launch_zero_hist(d_fd, (int)nf, st));
            base = 0;
            for (int gi = 0; gi < kGroups; ++gi) {
                const int nd = ndim_of(gi);
                if (!grp[gi].empty())
                    HIP_TRY(c, launch_compress_group(c, gi, d_fd + base, d_plan + base,
                                                     d_items + gi * (nf + 1), nitems[gi],
                                                     shape_for(c, 0, nd, max_R), max_R, st));
                base += (uint32_t)grp[gi].size();
            }
        }
    }
    std::unique_ptr<StageMark> cb_mark(given ? nullptr : new StageMark(c, SZ_STAGE_CODEBOOK, st));
    for (uint32_t k = 0; k < nf && !given; ++k)
        if (plans[k].status == -2)
            return fail(c, SZ_ERR_NONFINITE, "field %u holds %u non-finite values", perm[k],
                        plans[k].nonfinite);

    // host codebooks (Sec. VI-A), exact buffer sizes from the histogram;
    // with a given code book the words take their largest size and the
    // outlier lists a guess that the end checks
    auto outlier_guess = [](uint64_t n) { return std::min<uint64_t>(n, std::max<uint64_t>(n / 32, 4096)); };
    // the code books and tables of the fields are independent: a batch
    // spreads them over a few host threads (about 35 us each at 2R = 1024)
    std::vector<uint64_t> wbits(nf);
    auto make_codes = [&](uint32_t k) {
        const uint32_t i = perm[k];
        ResultInternal* R = ri(&res[i]);
        const int nsym = 2 * fds[k].R;
        if (given) {
            R->code_len.assign(given[i], given[i] + nsym);
        } else {
            R->plan = plans[k];
            R->code_len.assign(nsym, 0);
            huffman_lengths(hist[k].data(), nsym, kLmax, R->code_len.data());
        }
        uint8_t* h_len = reinterpret_cast<uint8_t*>(hs + o_cb[k]);
        uint32_t* h_cbook = reinterpret_cast<uint32_t*>(h_len + tables_len_bytes(nsym));
        std::memset(h_len, 0, tables_len_bytes(nsym));
        std::memcpy(h_len, R->code_len.data(), nsym);
        build_tables(R->code_len.data(), nsym, h_cbook, h_cbook + nsym);
        uint64_t bits = 0;
        if (given)
            bits = geo[i].npts * (uint64_t)kLmax;
        else
            for (int sy = 0; sy < nsym; ++sy) bits += (uint64_t)hist[k][sy] * R->code_len[sy];
        wbits[k] = bits;
    };
    if (nf >= 4) {   // a batch: the context's host workers join in
        if (!c->hpool) c->hpool.reset(new HostPool(7));
        const std::function<void(uint32_t)> f = make_codes;
        c->hpool->run(nf, f);
    } else {
        for (uint32_t k = 0; k < nf; ++k) make_codes(k);
    }
    for (uint32_t k = 0; k < nf; ++k) {
        const uint32_t i = perm[k];
        ResultInternal* R = ri(&res[i]);
        const int nsym = 2 * fds[k].R;
        const uint8_t* h_tabs = reinterpret_cast<const uint8_t*>(hs + o_cb[k]);
        const uint64_t nout = given ? outlier_guess(geo[i].npts) : hist[k][0];
        const uint64_t wcap = wbits[k] / 32 + geo[i].nchunks + 1;
        if ((s = res_alloc(c, R, wcap + kWordPad, &res[i].words))) return s;
        if ((s = res_alloc(c, R, (wcap + 31) / 32 + wcap, &R->d_esec))) return s;
        if ((s = res_alloc(c, R, std::max<uint64_t>(nout, 1), &res[i].outlier_idx))) return s;
        if ((s = res_alloc(c, R, std::max<uint64_t>(nout, 1), &res[i].outlier_val))) return s;
        res[i].n_outliers = nout;
        fds[k].words = res[i].words;
        fds[k].outlier_idx = res[i].outlier_idx;
        fds[k].outlier_val = res[i].outlier_val;
        fds[k].n_outliers = nout;
        fds[k].words_cap = wcap;
        fds[k].dtab = R->d_dtab;
        if (graphs)   // the result keeps its own histogram
            HIP_TRY(c, hipMemcpyAsync(res[i].hist, fds[k].hist, sizeof(uint32_t) * nsym,
                                      hipMemcpyDeviceToDevice, st));
        // lengths, codebook and decode tables in one copy (a batch's in one
        // copy for all fields and a scatter)
        fds[k].tab_src = o_cb[k] - o_cb[0];
        if (!many)
            HIP_TRY(c, hipMemcpyAsync(res[i].code_len, h_tabs, tables_bytes(nsym),
                                      hipMemcpyHostToDevice, st));
    }
    if (many)
        HIP_TRY(c, hipMemcpyAsync(d_scr + o_cb[0], hs + o_cb[0], o_cb[nf] - o_cb[0],
                                  hipMemcpyHostToDevice, st));
    std::vector<FieldDesc> hfd(nf);
    {
        uint64_t cb = 0;
        for (uint32_t j = 0; j < nf; ++j) {
            hfd[j] = fds[hord[j]];
            hfd[j].chunk_base = cb;
            hfd[j].nzw = d_fnz + j;
            cb += hfd[j].nchunks;
        }
    }
    // the elision's fields (encode order): words, section, the device word
    // offsets that bound them; tiles of each field's word capacity
    std::vector<ElideField> ef(nf);
    std::vector<uint64_t> etoff(nf + 1, 0);
    for (size_t g = 0; g < groups.size(); ++g)
        for (uint32_t j = groups[g].fs; j < groups[g].fe; ++j) {
            const uint64_t lo = gboff[gboff_at[g] + (j - groups[g].fs)];
            const uint64_t hi = gboff[gboff_at[g] + (j - groups[g].fs) + 1];
            ef[j].words = hfd[j].words;
            ef[j].sec = ri(&res[perm[hord[j]]])->d_esec;
            ef[j].wbeg = d_bwoff + goff_at[g] + lo;
            ef[j].wend = d_bwoff + goff_at[g] + hi;
            ef[j].nzw = d_fnz + j;
            ef[j].nw = 0;
        }
    for (uint32_t j = 0; j < nf; ++j)
        etoff[j + 1] = etoff[j] + (hfd[j].words_cap + etw - 1) / etw;
    const uint64_t etiles = etoff[nf];
    if (etiles > etiles_max) return fail(c, SZ_ERR_DEVICE, "elision tiles exceed their bound");
    // part 2: Huffman stats, block scans, encode with outlier compaction,
    // zero-word elision
    auto enqueue2 = [&](hipStream_t q) -> sz_status {
        for (size_t g = 0; g < groups.size(); ++g) {
            const uint32_t fs = groups[g].fs, nfg = groups[g].fe - groups[g].fs;
            const uint64_t b0 = hboff[fs], nb = hboff[groups[g].fe] - b0;
            const int chunk = hfd[fs].chunk;
            {
                STAGE(c, SZ_STAGE_HUFF_STATS, q);
                HIP_TRY(c, launch_huff_stats(d_hfd + fs, (int)nfg, d_gboff + gboff_at[g], nb, chunk,
                                             d_cwords, d_couts, d_bw + b0, d_bo + b0, 2 * max_R, q));
            }
            {
                STAGE(c, SZ_STAGE_SCAN, q);
                HIP_TRY(c, launch_scan_blocks(d_bw + b0, d_bo + b0, nb, d_bwoff + goff_at[g],
                                              d_booff + goff_at[g], q));
            }
            {
                STAGE(c, SZ_STAGE_ENCODE, q);
                HIP_TRY(c, launch_huff_encode(d_hfd + fs, (int)nfg, d_gboff + gboff_at[g], nb, chunk,
                                              d_cwords, d_couts, d_bwoff + goff_at[g],
                                              d_booff + goff_at[g], d_bnz + b0, 2 * max_R, q));
            }
        }
        {
            STAGE(c, SZ_STAGE_ELIDE, q);
            HIP_TRY(c, launch_elide(d_ef, (int)nf, d_etoff, etiles, etw, d_ecnt, d_eoff, 0, q));
        }
        return SZ_OK;
    };
    // sync 2: block word offsets and non-zero word counts (small) to the host
    std::vector<uint64_t> bwoff(nbw);
    std::vector<uint32_t> bnz(std::max<uint64_t>(total_blocks, 1));
    // with given code books, after the end: the plans and, where a field has
    // more outliers than its guessed lists hold, exact lists and the encode
    // again (eagerly, on the caller's stream)
    auto given_checks = [&](hipStream_t q) -> sz_status {
        for (uint32_t k = 0; k < nf; ++k) {
            if (plans[k].status == -2)
                return fail(c, SZ_ERR_NONFINITE, "field %u holds %u non-finite values", perm[k],
                            plans[k].nonfinite);
            ri(&res[perm[k]])->plan = plans[k];
        }
        bool again = false;
        for (uint32_t j = 0; j < nf; ++j) {
            const uint32_t k = hord[j], i = perm[k];
            const uint64_t nout = hist[k][0];
            if (nout > fds[k].n_outliers) {
                ResultInternal* R = ri(&res[i]);
                sz_status r;
                if ((r = res_alloc(c, R, nout, &res[i].outlier_idx))) return r;
                if ((r = res_alloc(c, R, nout, &res[i].outlier_val))) return r;
                fds[k].outlier_idx = hfd[j].outlier_idx = res[i].outlier_idx;
                fds[k].outlier_val = hfd[j].outlier_val = res[i].outlier_val;
                fds[k].n_outliers = hfd[j].n_outliers = nout;
                again = true;
            }
            res[i].n_outliers = nout;
        }
        if (again) {
            std::memcpy(hs + o_hfd, hfd.data(), sizeof(FieldDesc) * nf);
            HIP_TRY(c, hipMemcpyAsync(d_hfd, hs + o_hfd, sizeof(FieldDesc) * nf, hipMemcpyHostToDevice, q));
            sz_status r = enqueue2(q);
            if (r) return r;
            HIP_TRY(c, hipMemcpyAsync(hs + o_back, d_bwoff, n_back, hipMemcpyDeviceToHost, q));
            HIP_TRY(c, hipStreamSynchronize(q));
            std::memcpy(bwoff.data(), hs + o_bwoff, sizeof(uint64_t) * nbw);
            std::memcpy(bnz.data(), hs + o_bnz, sizeof(uint32_t) * total_blocks);
        }
        return SZ_OK;
    };
    if (graphs) {
        char* h = static_cast<char*>(c->parena);
        char* d = static_cast<char*>(c->arena);
        std::memcpy(h + o_hfd, hfd.data(), sizeof(FieldDesc) * nf);
        std::memcpy(h + o_gboff, gboff.data(), sizeof(uint64_t) * gboff.size());
        std::memcpy(h + o_ef, ef.data(), sizeof(ElideField) * nf);
        std::memcpy(h + o_etoff, etoff.data(), sizeof(uint64_t) * (nf + 1));
        std::vector<uint64_t> sig = {nf, groups.size(), total_blocks, total_chunks, (uint64_t)max_R, L.off,
                                     etiles};
        for (size_t g = 0; g < groups.size(); ++g) {
            sig.push_back(groups[g].fs);
            sig.push_back(groups[g].fe);
            sig.push_back((uint64_t)hfd[groups[g].fs].chunk);
            sig.push_back(hboff[groups[g].fe]);
        }
        cb_mark.reset();
        s = graph_run(c, 2, sig, o_hfd, end2 - o_hfd, st, [&](hipStream_t q) -> sz_status {
            sz_status r = enqueue2(q);
            if (r) return r;
            HIP_TRY(c, hipMemcpyAsync(h + o_bwoff, d + o_bwoff, sizeof(uint64_t) * nbw,
                                      hipMemcpyDeviceToHost, q));
            HIP_TRY(c, hipMemcpyAsync(h + o_bnz, d + o_bnz, sizeof(uint32_t) * total_blocks,
                                      hipMemcpyDeviceToHost, q));
            return SZ_OK;
        });
        if (s) return s;
        HIP_TRY(c, hipStreamSynchronize(c->gstream));
        HIP_TRY(c, hipStreamSynchronize(st));
        std::memcpy(bwoff.data(), h + o_bwoff, sizeof(uint64_t) * nbw);
        std::memcpy(bnz.data(), h + o_bnz, sizeof(uint32_t) * total_blocks);
        if (given) {
            std::memcpy(plans.data(), h + o_plan, sizeof(FieldPlan) * nf);
            for (uint32_t k = 0; k < nf; ++k)
                std::memcpy(hist[k].data(), h + o_hist + sizeof(uint32_t) * k * hstride,
                            sizeof(uint32_t) * hist[k].size());
            if ((s = given_checks(st))) return s;
        }
    } else {
        std::memcpy(hs + o_hfd, hfd.data(), sizeof(FieldDesc) * nf);
        std::memcpy(hs + o_gboff, gboff.data(), sizeof(uint64_t) * gboff.size());
        std::memcpy(hs + o_ef, ef.data(), sizeof(ElideField) * nf);
        std::memcpy(hs + o_etoff, etoff.data(), sizeof(uint64_t) * (nf + 1));
        HIP_TRY(c, hipMemcpyAsync(d_hfd, hs + o_hfd, end2 - o_hfd, hipMemcpyHostToDevice, st));
        if (many) HIP_TRY(c, launch_scatter_tables(d_hfd, (int)nf, reinterpret_cast<const uint8_t*>(d_scr + o_cb[0]), st));
        cb_mark.reset();
        if ((s = enqueue2(st))) return s;
        HIP_TRY(c, hipMemcpyAsync(hs + o_back, d_bwoff, n_back, hipMemcpyDeviceToHost, st));
        if (given && (s = read_plans_hists(st))) return s;
        HIP_TRY(c, hipStreamSynchronize(st));
        std::memcpy(bwoff.data(), hs + o_bwoff, sizeof(uint64_t) * nbw);
        std::memcpy(bnz.data(), hs + o_bnz, sizeof(uint32_t) * total_blocks);
        if (given) {
            std::memcpy(plans.data(), hs + o_plan, sizeof(FieldPlan) * nf);
            for (uint32_t k = 0; k < nf; ++k)
                std::memcpy(hist[k].data(), hs + o_hist + sizeof(uint32_t) * k * hstride,
                            sizeof(uint32_t) * hist[k].size());
            if ((s = given_checks(st))) return s;
        }
    }
    resolve_marks(c);
    for (size_t g = 0; g < groups.size(); ++g) {
        for (uint32_t j = groups[g].fs; j < groups[g].fe; ++j) {
            const uint64_t lo = gboff[gboff_at[g] + (j - groups[g].fs)];
            const uint64_t hi = gboff[gboff_at[g] + (j - groups[g].fs) + 1];
            const uint32_t k = hord[j];
            const uint32_t i = perm[k];
            res[i].n_words = bwoff[goff_at[g] + hi] - bwoff[goff_at[g] + lo];
            if (res[i].n_words > fds[k].words_cap)   // sized from the histogram or the largest
                return fail(c, SZ_ERR_DEVICE, "field %u: %llu Huffman words exceed the %llu sized "
                            "from the histogram", i, (unsigned long long)res[i].n_words,
                            (unsigned long long)fds[k].words_cap);
            uint64_t nz = 0;   // non-zero words of the field's encode blocks
            for (uint64_t b = hboff[j]; b < hboff[j + 1]; ++b) nz += bnz[b];
            ri(&res[i])->nzw = nz;
            if (!words_elided(&res[i], ri(&res[i]))) {   // the section buffer is not needed
                res_release(c, ri(&res[i]), ri(&res[i])->d_esec);
                ri(&res[i])->d_esec = nullptr;
            }
            res[i].compressed_bytes =
                blob_bytes(&res[i], fds[k].R, words_section_bytes(&res[i], ri(&res[i])));
            make_header(&res[i], ri(&res[i]), res[i].header);
        }
    }
    guard.keep = true;
    for (uint32_t i = 0; i < nf; ++i) outs[i] = res[i];
    return SZ_OK;
}

}  // namespace

extern "C" {

sz_status sz_compress_batch(sz_ctx* c, uint32_t nf, const float* const* d_in, const sz_dims* dims,
                            const sz_params* params, void* stream, sz_result* outs) {
    return compress_fields(c, nf, d_in, dims, params, nullptr, stream, outs);
}

sz_status sz_compress_batch_with_code(sz_ctx* c, uint32_t nf, const float* const* d_in,
                                      const sz_dims* dims, const sz_params* params,
                                      const uint8_t* const* code_len, void* stream, sz_result* outs) {
    if (!c) return SZ_ERR_INVALID_ARG;
    if (!code_len) return fail(c, SZ_ERR_INVALID_ARG, "null code books");
    return compress_fields(c, nf, d_in, dims, params, code_len, stream, outs);
}

sz_status sz_compress(sz_ctx* c, const float* d_in, const sz_dims* dims, const sz_params* params,
                      void* stream, sz_result* out) {
    if (!c) return SZ_ERR_INVALID_ARG;
    if (!out) return fail(c, SZ_ERR_INVALID_ARG, "null result");
    const float* ins[1] = {d_in};
    return compress_fields(c, 1, ins, dims, params, nullptr, stream, out);
}

sz_status sz_compress_with_code(sz_ctx* c, const float* d_in, const sz_dims* dims,
                                const sz_params* params, const uint8_t* code_len, void* stream,
                                sz_result* out) {
    if (!c) return SZ_ERR_INVALID_ARG;
    if (!out || !code_len) return fail(c, SZ_ERR_INVALID_ARG, "null result or code book");
    const float* ins[1] = {d_in};
    const uint8_t* lens[1] = {code_len};
    return compress_fields(c, 1, ins, dims, params, lens, stream, out);
}

sz_status sz_code_lengths(const uint32_t* hist, uint32_t nsym, uint8_t* code_len) {
    if (!hist || !code_len || nsym < 2 || nsym > 2 * (uint32_t)kMaxRadius)
        return SZ_ERR_INVALID_ARG;
    // every symbol counted once more, so that each gets a code
    std::vector<uint32_t> h(nsym);
    for (uint32_t s = 0; s < nsym; ++s) h[s] = hist[s] == UINT32_MAX ? hist[s] : hist[s] + 1u;
    huffman_lengths(h.data(), (int)nsym, kLmax, code_len);
    return SZ_OK;
}

sz_status sz_decompress_batch(sz_ctx* c, uint32_t nf, const sz_result* res, float* const* d_out,
                              void* stream) {
    if (!c) return SZ_ERR_INVALID_ARG;
    if (nf == 0 || !res || !d_out) return fail(c, SZ_ERR_INVALID_ARG, "empty batch or null argument");
    HIP_TRY(c, hipSetDevice(c->device));
    MarkGuard mark_guard{c};
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc(c);
    std::vector<FieldDesc> fds(nf);
    std::vector<FieldPlan> plans(nf);
    std::vector<uint32_t> grp[kGroups];
    std::vector<Geometry> geo(nf);
    int max_R = 0;
    for (uint32_t i = 0; i < nf; ++i) {
        const ResultInternal* R = ri(&res[i]);
        if (!R || !d_out[i] || !res[i].words || !res[i].chunk_bits || !res[i].anchors)
            return fail(c, SZ_ERR_INVALID_ARG, "result %u is empty or output is null", i);
        if (reinterpret_cast<uintptr_t>(d_out[i]) & 3u)
            return fail(c, SZ_ERR_INVALID_ARG, "output %u not 4-byte aligned", i);
        sz_params p;
        sz_params_default(&p);
        p.radius = (uint32_t)R->R;
        p.huff_chunk = (uint32_t)R->chunk;
        p.eb_mode = R->eb_mode;
        p.eb = R->eb >= 0 ? R->eb : 0;
        p.anchor_stride = (uint32_t)R->S;
        for (int k = 0; k < (int)R->dims.ndim && k < 3; ++k) p.window[k] = (uint32_t)R->w[k];
        sz_status s = check_field(c, &R->dims, &p, geo[i]);
        if (s) return s;
        if (res[i].n != geo[i].npts || res[i].n_chunks != geo[i].nchunks ||
            res[i].n_anchors != geo[i].nanch)
            return fail(c, SZ_ERR_CORRUPT, "result %u: sizes do not match its dimensions", i);
        grp[group_of(geo[i])].push_back(i);
        max_R = std::max(max_R, geo[i].R);
    }
    std::vector<uint32_t> perm;
    for (int gi = 0; gi < kGroups; ++gi) perm.insert(perm.end(), grp[gi].begin(), grp[gi].end());
    uint64_t cb = 0;
    bool split = true;   // every field has sub-chunk offsets: kSubParts decode lanes per chunk
    std::vector<uint64_t> dboff(nf + 1, 0);
    for (uint32_t k = 0; k < nf; ++k) {
        const uint32_t i = perm[k];
        const ResultInternal* R = ri(&res[i]);
        FieldDesc& f = fds[k];
        sz_params p;
        sz_params_default(&p);
        fill_desc(geo[i], &p, f);
        f.out = d_out[i];
        f.anchors = res[i].anchors;
        f.words = res[i].words;
        f.chunk_bits = res[i].chunk_bits;
        f.sub = R->d_sub;
        split = split && R->d_sub != nullptr;
        f.outlier_idx = res[i].outlier_idx;
        f.outlier_val = res[i].outlier_val;
        f.n_outliers = res[i].n_outliers;
        f.words_cap = res[i].n_words;
        f.dtab = R->d_dtab;
        f.chunk_base = cb;
        uint16_t* codes;
        sz_status s = sc.get(geo[i].npts, &codes);
        if (s) return s;
        f.codes = codes;
        cb += geo[i].nchunks;
        dboff[k + 1] = dboff[k] + (geo[i].nchunks + kDecBlockChunks - 1) / kDecBlockChunks;
        plans[k] = R->plan;
    }
    std::vector<uint64_t> items(kGroups * (nf + 1), 0);
    uint64_t nitems[kGroups] = {0, 0, 0, 0};
    for (int gi = 0; gi < kGroups; ++gi) {
        uint64_t* io = items.data() + gi * (nf + 1);
        for (size_t j = 0; j < grp[gi].size(); ++j)
            io[j + 1] = io[j] + (geo[grp[gi][j]].nwin_total + kWinPerGroup - 1) / kWinPerGroup;
        nitems[gi] = grp[gi].empty() ? 0 : io[grp[gi].size()];
    }
    const uint64_t nblocks = dboff[nf];
    FieldDesc* d_fd;
    FieldPlan* d_plan;
    uint64_t *d_items, *d_dboff;
    uint32_t* d_bsum;
    sz_status s;
    // the device work of the call
    auto enqueue = [&](hipStream_t q) -> sz_status {
        {
            // block word counts, the outlier scatter and the pass descriptors
            STAGE(c, SZ_STAGE_SCAN, q);
            HIP_TRY(c, launch_dec_prep(d_fd, d_plan, (int)nf, d_dboff, nblocks, d_bsum, q));
        }
        {
            STAGE(c, SZ_STAGE_DECODE, q);
            HIP_TRY(c, launch_huff_decode(d_fd, (int)nf, d_dboff, nblocks, d_bsum, 2 * max_R,
                                          split ? 1 : 0, q));
        }
        uint32_t base = 0;
        for (int gi = 0; gi < kGroups; ++gi) {
            if (!grp[gi].empty()) {
                STAGE(c, SZ_STAGE_REPLAY, q);
                HIP_TRY(c, launch_decompress_group(c, gi, d_fd + base, d_plan + base,
                                                   d_items + gi * (nf + 1), nitems[gi],
                                                   shape_for(c, 1, ndim_of(gi), max_R), q));
            }
            base += (uint32_t)grp[gi].size();
        }
        return SZ_OK;
    };
    if (c->graphs) {
        Layout L;
        const size_t o_fd = L.take<FieldDesc>(nf), o_plan = L.take<FieldPlan>(nf);
        const size_t o_items = L.take<uint64_t>(items.size()), o_dboff = L.take<uint64_t>(nf + 1);
        const size_t staged = L.off;
        const size_t o_bsum = L.take<uint32_t>(std::max<uint64_t>(nblocks, 1));
        if ((s = arena_reserve(c, L.off))) return s;
        char* h = static_cast<char*>(c->parena);
        char* d = static_cast<char*>(c->arena);
        std::memcpy(h + o_fd, fds.data(), sizeof(FieldDesc) * nf);
        std::memcpy(h + o_plan, plans.data(), sizeof(FieldPlan) * nf);
        std::memcpy(h + o_items, items.data(), sizeof(uint64_t) * items.size());
        std::memcpy(h + o_dboff, dboff.data(), sizeof(uint64_t) * (nf + 1));
        d_fd = reinterpret_cast<FieldDesc*>(d + o_fd);
        d_plan = reinterpret_cast<FieldPlan*>(d + o_plan);
        d_items = reinterpret_cast<uint64_t*>(d + o_items);
        d_dboff = reinterpret_cast<uint64_t*>(d + o_dboff);
        d_bsum = reinterpret_cast<uint32_t*>(d + o_bsum);
        // everything the launches' arguments depend on
        const LaunchShape s3 = shape_for(c, 1, 3, max_R), s2 = shape_for(c, 1, 2, max_R);
        const std::vector<uint64_t> sig = {nf, nblocks, nitems[0], nitems[1], nitems[2], nitems[3],
                                           grp[0].size(), grp[1].size(), grp[2].size(),
                                           (uint64_t)max_R, (uint64_t)s3.per_cu, (uint64_t)s2.variant,
                                           (uint64_t)s2.per_cu, L.off, split ? 1u : 0u};
        if ((s = graph_run(c, 0, sig, 0, staged, st, enqueue))) return s;
        HIP_TRY(c, hipStreamSynchronize(c->gstream));
        return SZ_OK;
    }
    // descriptors staged in pinned memory and sent in one asynchronous copy
    // to one scratch block of the same layout
    {
        Layout L;
        const size_t o_fd = L.take<FieldDesc>(nf), o_plan = L.take<FieldPlan>(nf);
        const size_t o_items = L.take<uint64_t>(items.size()), o_dboff = L.take<uint64_t>(nf + 1);
        const size_t staged = L.off;
        const size_t o_bsum = L.take<uint32_t>(std::max<uint64_t>(nblocks, 1));
        char* d;
        if ((s = sc.get(L.off, &d))) return s;
        if ((s = pinned_reserve(c, staged))) return s;
        d_fd = reinterpret_cast<FieldDesc*>(d + o_fd);
        d_plan = reinterpret_cast<FieldPlan*>(d + o_plan);
        d_items = reinterpret_cast<uint64_t*>(d + o_items);
        d_dboff = reinterpret_cast<uint64_t*>(d + o_dboff);
        d_bsum = reinterpret_cast<uint32_t*>(d + o_bsum);
        char* h = static_cast<char*>(c->pinned);
        std::memcpy(h + o_fd, fds.data(), sizeof(FieldDesc) * nf);
        std::memcpy(h + o_plan, plans.data(), sizeof(FieldPlan) * nf);
        std::memcpy(h + o_items, items.data(), sizeof(uint64_t) * items.size());
        std::memcpy(h + o_dboff, dboff.data(), sizeof(uint64_t) * (nf + 1));
        HIP_TRY(c, hipMemcpyAsync(d, h, staged, hipMemcpyHostToDevice, st));
    }
    if ((s = enqueue(st))) return s;
    // launch-shape tuning: the replay rewrites the same values
    uint32_t base = 0;
    for (int gi = 0; gi < kGroups; ++gi) {
        const int nd = ndim_of(gi);
        if (!grp[gi].empty() && tunable(gi) && needs_tuning(c, 1, nd, max_R)) {
            LaunchShape best;
            s = tune_shapes(c, nd, st, &best, [&](LaunchShape sh) -> sz_status {
                HIP_TRY(c, launch_decompress(nd, d_fd + base, d_plan + base, d_items + gi * (nf + 1),
                                             nitems[gi], c->num_cus, sh, st));
                return SZ_OK;
            });
            if (s) return s;
            c->shapes[{1, nd, max_R}] = best;
        }
        base += (uint32_t)grp[gi].size();
    }
    HIP_TRY(c, hipStreamSynchronize(st));
    resolve_marks(c);
    return SZ_OK;
}

sz_status sz_decompress(sz_ctx* c, const sz_result* res, float* d_out, void* stream) {
    if (!c) return SZ_ERR_INVALID_ARG;
    float* outs[1] = {d_out};
    return sz_decompress_batch(c, 1, res, outs, stream);
}

// One field, decompressed with the static workspace only: the same kernels
// as sz_decompress, launched with their default shapes; nothing is
// allocated, nothing waits for the stream.
sz_status sz_decompress_noalloc(sz_ctx* c, const sz_result* res, float* d_out, void* stream) {
    if (!c) return SZ_ERR_INVALID_ARG;
    if (!res || !d_out) return fail(c, SZ_ERR_INVALID_ARG, "null result or output");
    if (reinterpret_cast<uintptr_t>(d_out) & 3u)
        return fail(c, SZ_ERR_INVALID_ARG, "output not 4-byte aligned");
    if (!c->noalloc) return fail(c, SZ_ERR_DEVICE, "no workspace on device %d", c->device);
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const ResultInternal* R = ri(res);
    if (!R || !res->words || !res->chunk_bits || !res->anchors)
        return fail(c, SZ_ERR_INVALID_ARG, "the result is empty");
    sz_params p;
    sz_params_default(&p);
    p.radius = (uint32_t)R->R;
    p.huff_chunk = (uint32_t)R->chunk;
    p.eb_mode = R->eb_mode;
    p.eb = R->eb >= 0 ? R->eb : 0;
    p.anchor_stride = (uint32_t)R->S;
    for (int k = 0; k < (int)R->dims.ndim && k < 3; ++k) p.window[k] = (uint32_t)R->w[k];
    Geometry geo;
    sz_status s = check_field(c, &R->dims, &p, geo);
    if (s) return s;
    if (res->n != geo.npts || res->n_chunks != geo.nchunks || res->n_anchors != geo.nanch)
        return fail(c, SZ_ERR_CORRUPT, "sizes do not match the dimensions");
    if (geo.npts > kNoAllocMaxPoints)
        return fail(c, SZ_ERR_UNSUPPORTED,
                    "%llu points: the workspace of sz_decompress_noalloc holds fields of up to "
                    "%llu points",
                    (unsigned long long)geo.npts, (unsigned long long)kNoAllocMaxPoints);
    // workspace layout: descriptors (staged by one kernel), block word
    // counts, decoded quant-codes
    FieldDesc f;
    fill_desc(geo, &p, f);
    const uint64_t nblocks = (geo.nchunks + kDecBlockChunks - 1) / kDecBlockChunks;
    const uint64_t ngroups = (geo.nwin_total + kWinPerGroup - 1) / kWinPerGroup;
    Layout L;
    const size_t o_fd = L.take<FieldDesc>(1), o_plan = L.take<FieldPlan>(1);
    const size_t o_items = L.take<uint64_t>(2), o_dboff = L.take<uint64_t>(2);
    const size_t staged = L.off;
    const size_t o_bsum = L.take<uint32_t>(nblocks), o_codes = L.take<uint16_t>(geo.npts);
    if (L.off > kNoAllocScratchBytes || staged > sizeof(uint32_t) * kStageWordsMax)
        return fail(c, SZ_ERR_UNSUPPORTED, "workspace of %llu bytes needed",
                    (unsigned long long)L.off);
    char* ws = static_cast<char*>(c->noalloc);
    f.out = d_out;
    f.anchors = res->anchors;
    f.words = res->words;
    f.chunk_bits = res->chunk_bits;
    f.sub = R->d_sub;
    f.outlier_idx = res->outlier_idx;
    f.outlier_val = res->outlier_val;
    f.n_outliers = res->n_outliers;
    f.words_cap = res->n_words;
    f.dtab = R->d_dtab;
    f.chunk_base = 0;
    f.codes = reinterpret_cast<uint16_t*>(ws + o_codes);
    StageWords sw;
    std::memset(&sw, 0, sizeof sw);
    sw.n = (uint32_t)((staged + 3) / 4);
    char* sb = reinterpret_cast<char*>(sw.w);
    const uint64_t items[2] = {0, ngroups}, dboff[2] = {0, nblocks};
    std::memcpy(sb + o_fd, &f, sizeof f);
    std::memcpy(sb + o_plan, &R->plan, sizeof(FieldPlan));
    std::memcpy(sb + o_items, items, sizeof items);
    std::memcpy(sb + o_dboff, dboff, sizeof dboff);
    FieldDesc* d_fd = reinterpret_cast<FieldDesc*>(ws + o_fd);
    FieldPlan* d_plan = reinterpret_cast<FieldPlan*>(ws + o_plan);
    const uint64_t* d_items = reinterpret_cast<const uint64_t*>(ws + o_items);
    const uint64_t* d_dboff = reinterpret_cast<const uint64_t*>(ws + o_dboff);
    uint32_t* d_bsum = reinterpret_cast<uint32_t*>(ws + o_bsum);
    HIP_TRY(c, launch_stage_words(reinterpret_cast<uint32_t*>(ws), sw, st));
    HIP_TRY(c, launch_dec_prep(d_fd, d_plan, 1, d_dboff, nblocks, d_bsum, st));
    HIP_TRY(c, launch_huff_decode(d_fd, 1, d_dboff, nblocks, d_bsum, 2 * geo.R,
                                  R->d_sub != nullptr ? 1 : 0, st));
    HIP_TRY(c, launch_decompress_group(c, group_of(geo), d_fd, d_plan, d_items, ngroups,
                                       shape_for(c, 1, geo.ndim, geo.R), st));
    return SZ_OK;
}

sz_status sz_result_free(sz_ctx* c, sz_result* r) {
    if (!c || !r) return SZ_ERR_INVALID_ARG;
    release_result(c, r);
    return SZ_OK;
}

sz_status sz_result_read(sz_ctx* c, const sz_result* r, int32_t section, void* dst, uint64_t cap,
                         uint64_t* written) {
    if (!c || !r || !r->internal) return fail(c, SZ_ERR_INVALID_ARG, "empty result");
    const ResultInternal* R = ri(r);
    const void* src = nullptr;
    uint64_t bytes = 0;
    switch (section) {
    case SZ_SEC_ANCHORS: src = r->anchors; bytes = r->n_anchors * 4; break;
    case SZ_SEC_CODES: src = r->codes; bytes = r->codes ? r->n * 2 : 0; break;
    case SZ_SEC_OUTLIER_IDX: src = r->outlier_idx; bytes = r->n_outliers * 4; break;
    case SZ_SEC_OUTLIER_VAL: src = r->outlier_val; bytes = r->n_outliers * 4; break;
    case SZ_SEC_WORDS: src = r->words; bytes = r->n_words * 4; break;
    case SZ_SEC_CHUNK_BITS: src = r->chunk_bits; bytes = r->n_chunks * 2; break;
    case SZ_SEC_HIST: src = r->hist; bytes = r->hist ? (uint64_t)2 * R->R * 4 : 0; break;
    case SZ_SEC_CODE_LEN: src = r->code_len; bytes = (uint64_t)2 * R->R; break;
    default: return fail(c, SZ_ERR_INVALID_ARG, "section %d", section);
    }
    if (written) *written = bytes;
    if (bytes > cap) return fail(c, SZ_ERR_CAPACITY, "section needs %llu bytes", (unsigned long long)bytes);
    if (bytes == 0) return SZ_OK;
    if (!dst) return fail(c, SZ_ERR_INVALID_ARG, "null destination");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    return SZ_OK;
}

sz_status sz_serialize(sz_ctx* c, const sz_result* r, void* dst, uint64_t cap, uint64_t* written) {
    if (!c || !r || !r->internal) return fail(c, SZ_ERR_INVALID_ARG, "empty result");
    const ResultInternal* R = ri(r);
    const uint64_t total = blob_bytes(r, R->R, words_section_bytes(r, R));
    if (written) *written = total;
    if (cap < total) return fail(c, SZ_ERR_CAPACITY, "blob needs %llu bytes", (unsigned long long)total);
    if (!dst) return fail(c, SZ_ERR_INVALID_ARG, "null destination");
    HIP_TRY(c, hipSetDevice(c->device));
    uint8_t* out = static_cast<uint8_t*>(dst);
    std::memset(out, 0, total);
    uint8_t* h = out;
    make_header(r, R, h);
    struct Sec {
        const void* src;
        uint64_t bytes;
    } secs[6] = {{r->anchors, r->n_anchors * 4},   {r->code_len, (uint64_t)2 * R->R},
                 {r->chunk_bits, r->n_chunks * 2}, {r->words, r->n_words * 4},
                 {r->outlier_idx, r->n_outliers * 4}, {r->outlier_val, r->n_outliers * 4}};
    uint64_t pos = 256;
    for (int k = 0; k < 6; ++k) {
        if (k == 3 && words_elided(r, R)) {
            // the words without their zero words, as the compression built
            // them on the device: bitmap, then the others
            if (!R->d_esec) return fail(c, SZ_ERR_INVALID_ARG, "no elided words section");
            const uint64_t nsec = elided_words(r->n_words, R->nzw);
            HIP_TRY(c, hipMemcpy(out + pos, R->d_esec, nsec * 4, hipMemcpyDeviceToHost));
            put32(h, 224 + 4 * k, crc32_update(0, out + pos, nsec * 4));
            pos += pad8(nsec * 4);
            continue;
        }
        if (secs[k].bytes) HIP_TRY(c, hipMemcpy(out + pos, secs[k].src, secs[k].bytes, hipMemcpyDeviceToHost));
        put32(h, 224 + 4 * k, crc32_update(0, out + pos, secs[k].bytes));
        pos += pad8(secs[k].bytes);
    }
    put32(h, 252, crc32_update(0, h, 252));
    return SZ_OK;
}

sz_status sz_upload(sz_ctx* c, const void* blob, uint64_t bytes, void* stream, sz_result* out) {
    if (!c) return SZ_ERR_INVALID_ARG;
    if (!blob || !out) return fail(c, SZ_ERR_INVALID_ARG, "null argument");
    const uint8_t* b = static_cast<const uint8_t*>(blob);
    BlobInfo bi;
    {
        std::string why;
        const sz_status s = parse_blob(b, bytes, &bi, &why);
        if (s) return fail(c, s, "%s", why.c_str());
    }
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Geometry& g = bi.geo;
    const bool elided = bi.elided;
    const uint64_t wsec = bi.wsec;
    const uint64_t* off = bi.off;
    const uint64_t* secb = bi.secb;
    const int nsym = 2 * g.R;
    sz_status s;
    sz_result r;
    std::memset(&r, 0, sizeof r);
    r.n = g.npts;
    r.n_anchors = bi.n_anchors;
    r.n_chunks = bi.n_chunks;
    r.n_words = bi.n_words;
    r.n_outliers = bi.n_outliers;
    ResultInternal* R = new ResultInternal();
    R->owner = c;
    r.internal = R;
    R->dims = bi.dims;
    R->S = g.S;
    for (int k = 0; k < 3; ++k) R->w[k] = g.w[k];
    R->R = g.R;
    R->chunk = g.chunk;
    R->eb_mode = bi.params.eb_mode;
    R->eb = bi.params.eb;
    R->nzw = bi.nzw;
    R->code_len.assign(b + off[1], b + off[1] + nsym);
    std::memset(&R->plan, 0, sizeof R->plan);
    R->plan.alpha = bi.alpha;
    R->plan.vmin = bi.vmin;
    R->plan.vmax = bi.vmax;
    R->plan.e = bi.e;
    R->plan.levels = g.L;
    for (int l = 0; l < g.L; ++l) {
        R->plan.el[l] = bi.el[l];
        R->plan.ebx2[l] = 2.0f * R->plan.el[l];
    }
    for (int k = 0; k < 3; ++k) {
        R->plan.spline[k] = bi.spline[k];
        R->plan.order[k] = bi.order[k];
    }
    std::vector<uint32_t> cbook(nsym), dtab(dtab_words(nsym));
    build_tables(R->code_len.data(), nsym, cbook.data(), dtab.data());
    if ((s = res_alloc(c, R, r.n_anchors, &r.anchors)) || (s = res_alloc(c, R, nsym, &r.code_len)) ||
        (s = res_alloc(c, R, std::max<uint64_t>(r.n_chunks, 1), &r.chunk_bits)) ||
        (s = res_alloc(c, R, r.n_words + kWordPad, &r.words)) ||
        (elided && (s = res_alloc(c, R, wsec, &R->d_esec))) ||
        (s = res_alloc(c, R, std::max<uint64_t>(r.n_outliers, 1), &r.outlier_idx)) ||
        (s = res_alloc(c, R, std::max<uint64_t>(r.n_outliers, 1), &r.outlier_val)) ||
        (s = res_alloc(c, R, nsym, &R->d_cbook)) || (s = res_alloc(c, R, dtab.size(), &R->d_dtab))) {
        release_result(c, &r);
        return s;
    }
    void* dsts[6] = {r.anchors, r.code_len, r.chunk_bits, elided ? (void*)R->d_esec : (void*)r.words,
                     r.outlier_idx, r.outlier_val};
    for (int k = 0; k < 6; ++k)
        if (secb[k]) {
            hipError_t e = hipMemcpyAsync(dsts[k], b + off[k], secb[k], hipMemcpyHostToDevice, st);
            if (e != hipSuccess) {
                release_result(c, &r);
                return fail(c, SZ_ERR_DEVICE, "upload copy: %s", hipGetErrorString(e));
            }
        }
    Scratch sc(c);
    if (elided && r.n_words) {
        // the words from the elided section, on the device
        ElideField e;
        e.words = r.words;
        e.sec = R->d_esec;
        e.wbeg = e.wend = nullptr;
        e.nzw = nullptr;
        e.nw = r.n_words;
        const uint64_t tw = elide_tile_words(r.n_words);
        const uint64_t tiles = (r.n_words + tw - 1) / tw;
        const uint64_t toff[2] = {0, tiles};
        char* d;
        Layout L;
        const size_t o_e = L.take<ElideField>(1), o_t = L.take<uint64_t>(2);
        const size_t o_c = L.take<uint32_t>(tiles), o_o = L.take<uint64_t>(tiles + 1);
        if ((s = sc.get(L.off, &d))) {
            release_result(c, &r);
            return s;
        }
        hipError_t e1 = hipMemcpyAsync(d + o_e, &e, sizeof e, hipMemcpyHostToDevice, st);
        hipError_t e2 = hipMemcpyAsync(d + o_t, toff, sizeof toff, hipMemcpyHostToDevice, st);
        hipError_t e3 = hipSuccess;
        if (e1 == hipSuccess && e2 == hipSuccess) {
            STAGE(c, SZ_STAGE_ELIDE, st);
            e3 = launch_elide(reinterpret_cast<ElideField*>(d + o_e), 1,
                              reinterpret_cast<uint64_t*>(d + o_t), tiles, tw,
                              reinterpret_cast<uint32_t*>(d + o_c), reinterpret_cast<uint64_t*>(d + o_o),
                              1, st);
        }
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            release_result(c, &r);
            return fail(c, SZ_ERR_DEVICE, "upload: restoring the elided words failed");
        }
    }
    hipError_t e1 = hipMemcpyAsync(R->d_cbook, cbook.data(), 4 * nsym, hipMemcpyHostToDevice, st);
    hipError_t e2 = hipMemcpyAsync(R->d_dtab, dtab.data(), 4 * dtab.size(), hipMemcpyHostToDevice, st);
    hipError_t e3 = hipStreamSynchronize(st);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        release_result(c, &r);
        return fail(c, SZ_ERR_DEVICE, "upload copy failed");
    }
    std::memcpy(r.header, b, 256);
    r.compressed_bytes = bytes;
    *out = r;
    return SZ_OK;
}

// ------------------------------------------------------------ serving
sz_status sz_server_create(sz_server** out, int device, int slots, uint64_t hbm_budget_bytes) {
    if (!out || slots < 1 || slots > 64) return SZ_ERR_INVALID_ARG;
    *out = nullptr;
    sz_server* s = new sz_server();
    s->device = device;
    s->budget = hbm_budget_bytes;
    for (int i = 0; i < slots; ++i) {
        sz_ctx* c = nullptr;
        sz_status rc = sz_ctx_create(&c, device, 0);
        hipStream_t st = nullptr;
        if (rc == SZ_OK && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            sz_ctx_destroy(c);
            rc = SZ_ERR_DEVICE;
        }
        if (rc != SZ_OK) {
            for (size_t k = 0; k < s->ctx.size(); ++k) {
                (void)hipStreamDestroy(s->st[k]);
                sz_ctx_destroy(s->ctx[k]);
            }
            delete s;
            return rc;
        }
        s->ctx.push_back(c);
        s->st.push_back(st);
    }
    if (s->budget) {
        // the workers' caches count against the budget together with what
        // they hold; a worker returns cached blocks before passing it
        s->shared.reset(new SharedHeld());
        s->shared->budget = s->budget;
        s->shared->ctx = s->ctx;
        for (sz_ctx* c : s->ctx) c->shared = s->shared.get();
    }
    for (int i = 0; i < slots; ++i) s->th.emplace_back(server_worker, s, i);
    *out = s;
    return SZ_OK;
}

sz_status sz_server_submit(sz_server* s, const sz_request* req) {
    if (!s || !req) return SZ_ERR_INVALID_ARG;
    if (req->kind == SZ_REQ_COMPRESS ? (!req->d_in || req->book < 0)
                                     : (req->kind != SZ_REQ_DECOMPRESS || !req->src ||
                                        !req->src->internal || !req->d_out))
        return SZ_ERR_INVALID_ARG;
    const uint64_t need = request_need(*req);
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stop) return SZ_ERR_INVALID_ARG;
    if (s->budget && need > s->budget) {
        s->err = "request needs more device memory than the whole budget";
        return SZ_ERR_OOM;
    }
    s->q.push_back({*req, need, s->now()});
    s->cv_work.notify_one();
    return SZ_OK;
}

sz_status sz_server_poll(sz_server* s, sz_completion* out, uint32_t cap, uint32_t* n, int wait) {
    if (!s || !n || (cap && !out)) return SZ_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->m);
    if (wait)
        s->cv_done.wait(lk, [&] {
            return !s->done.empty() || (s->running == 0 && (s->q.empty() || admissible(s) < 0));
        });
    uint32_t k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return SZ_OK;
}

sz_status sz_server_result_free(sz_server* s, sz_result* res) {
    if (!s || !res || !res->internal) return SZ_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->m);
        auto it = s->held.find(res->internal);
        if (it == s->held.end()) return SZ_ERR_INVALID_ARG;
        s->charged -= it->second;
        s->held.erase(it);
    }
    release_result(ri(res)->owner, res);
    std::memset(res, 0, sizeof *res);
    s->cv_work.notify_all();
    return SZ_OK;
}

sz_status sz_server_stats(sz_server* s, uint64_t* charged, uint64_t* queued, uint64_t* running) {
    if (!s) return SZ_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->m);
    if (charged) *charged = s->charged;
    if (queued) *queued = s->q.size();
    if (running) *running = (uint64_t)s->running;
    return SZ_OK;
}

const char* sz_server_last_error(const sz_server* s) { return s ? s->err.c_str() : ""; }

sz_status sz_server_destroy(sz_server* s) {
    if (!s) return SZ_OK;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
        s->q.clear();   // requests not yet started are cancelled
    }
    s->cv_work.notify_all();
    for (auto& t : s->th) t.join();   // running requests finish
    for (auto& cp : s->done)
        if (cp.result.internal) {
            s->held.erase(cp.result.internal);
            release_result(ri(&cp.result)->owner, &cp.result);
        }
    // results the caller did not free: their blocks go with the contexts
    for (auto& kv : s->held) delete static_cast<ResultInternal*>(kv.first);
    for (size_t k = 0; k < s->ctx.size(); ++k) {
        (void)hipStreamDestroy(s->st[k]);
        sz_ctx_destroy(s->ctx[k]);
    }
    delete s;
    return SZ_OK;
}

}  // extern "C"
