// Host runtime and C ABI of libcdc (see include/cdc.h for the contract).
//
// The runtime plans a call (segment length, cut slots per segment, MAXP
// block length), carves the per-(device, stream) workspace and enqueues the
// kernel sequence.  It never synchronises except to grow a workspace, which
// it refuses to do while the stream is being captured.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "cdc.h"
#include "cdc_internal.h"
#include "stream.h"

namespace cdc {
namespace {

thread_local std::string t_last_error;

void set_error(const char* what, hipError_t e) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    t_last_error = buf;
}

// Tuning (speed only; never changes the offsets).  0 = built-in choice.
uint64_t g_chain_segment = 0;
uint64_t g_maxp_segment = 0;
int g_waves_per_block = 4;

constexpr uint64_t kMinSeg = 64 << 10;
// Segments and chunks are at most 2^28 bytes: the chain kernels keep
// positions as 32-bit offsets from the segment start.
constexpr uint64_t kMaxSeg = 1ull << 28;
constexpr uint64_t kMaxChunkLimit = 1ull << 28;
// RAM / AE: few long segments, so that speculated chains rejoin the true
// chain inside their segment; MAXP has no chain to rejoin (its candidates do
// not depend on the chunk start) and splits finely for load balance.
constexpr uint64_t kChainSegment = 512 << 10;
constexpr uint64_t kMaxpSegment = 256 << 10;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Event pairs around kernels, resolved when the caller asks for them.
struct EventMarks : Marks {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    int level = 0;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    bool open = false;

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin(const char* name, int lvl, hipStream_t st) override {
        open = false;
        if (lvl > level) return;
        hipEvent_t a = get(), b = get();
        if (!a || !b) return;
        (void)hipEventRecord(a, st);
        recs.push_back({name, a, b});
        open = true;
    }
    void end(int lvl, hipStream_t st) override {
        if (lvl > level || !open) return;
        (void)hipEventRecord(recs.back().b, st);
        open = false;
    }
};

int g_profile_level = 0;

// Streams of a workspace for running the algorithms of a batch side by
// side: RAM stays on the caller's stream, AE and AE-Min go to one side
// stream, MAXP to the other; they are forked from and joined back into the
// caller's stream by events (under capture this becomes parallel branches
// of the graph).  Two, so that with the caller's stream they fit the few
// hardware queues a process gets.  Default priority, non-blocking.
constexpr int kSide = 2;

struct SideStreams {
    bool ok = false;
    hipStream_t s[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};

    bool create() {
        for (int i = 0; i < kSide; i++)
            if (hipStreamCreateWithFlags(&s[i], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&join[i], hipEventDisableTiming) != hipSuccess)
                return false;
        if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess)
            return false;
        ok = true;
        return true;
    }
    void destroy() {
        for (int i = 0; i < kSide; i++) {
            if (s[i]) {
                (void)hipStreamSynchronize(s[i]);
                (void)hipStreamDestroy(s[i]);
            }
            if (join[i]) (void)hipEventDestroy(join[i]);
            s[i] = nullptr;
            join[i] = nullptr;
        }
        if (fork) (void)hipEventDestroy(fork);
        fork = nullptr;
        ok = false;
    }
};

struct Workspace {
    EventMarks marks;
    void* dev = nullptr;
    size_t cap = 0;
    // Buffers replaced by a larger one.  A HIP graph captured earlier on the
    // stream holds their addresses in its kernel arguments, so they stay
    // allocated until cdc_release (or until the stream's workspace is
    // dropped); growth is geometric, which bounds what they add up to.
    std::vector<void*> retired;
    // the last single RAM / AE call on the stream (for cdc_walk_stats)
    size_t last_meta = 0;
    uint32_t last_items = 0;
    // reservation for batches
    uint32_t res_jobs = 0;
    BatchCaps res_caps{};
    SideStreams side;
};

std::mutex g_mu;
std::map<std::pair<int, uintptr_t>, Workspace> g_ws;

}  // namespace

static int batch_on(Workspace& ws, const cdc_job* jobs, uint32_t n_jobs,
                    uint64_t bytes_hint, bool side, hipStream_t stream,
                    uint32_t algo_mask, uint64_t ram_max_n = ~0ull);

namespace {

Workspace& workspace_for(hipStream_t st) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    return g_ws[{dev, (uintptr_t)st}];
}

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

// Grow the workspace to `need` bytes.  Needs the stream idle: the old buffer
// may still be in use by work enqueued earlier.
int ensure(Workspace& ws, size_t need, hipStream_t st) {
    if (ws.cap >= need) return CDC_OK;
    if (capturing(st)) {
        t_last_error = "workspace must grow during stream capture; call cdc_reserve first";
        return CDC_ENOMEM;
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) { set_error("hipStreamSynchronize", e); return CDC_EHIP; }
    size_t cap = align_up(std::max(need, (size_t)1 << 20), (size_t)1 << 20);
    if (ws.dev) {
        cap = std::max(cap, align_up(ws.cap + ws.cap / 2, (size_t)1 << 20));
        ws.retired.push_back(ws.dev);
        ws.dev = nullptr;
        ws.cap = 0;
    }
    e = hipMalloc(&ws.dev, cap);
    if (e != hipSuccess) { set_error("hipMalloc workspace", e); return CDC_ENOMEM; }
    ws.cap = cap;
    // the error word lives at offset 0 and starts cleared
    e = hipMemsetAsync(ws.dev, 0, 256, st);
    if (e != hipSuccess) { set_error("hipMemsetAsync", e); return CDC_EHIP; }
    return CDC_OK;
}

bool params_valid(uint32_t algo, uint32_t w, uint32_t M) {
    return algo <= 3 && w >= 1 && (uint64_t)M >= (uint64_t)w + 1 &&
           (uint64_t)M <= kMaxChunkLimit;
}

uint64_t chain_segment() { return g_chain_segment ? g_chain_segment : kChainSegment; }
uint64_t maxp_segment() { return g_maxp_segment ? g_maxp_segment : kMaxpSegment; }

uint64_t choose_segment(uint32_t algo, uint64_t n) {
    (void)n;
    return algo == kMaxp ? maxp_segment() : chain_segment();
}

uint32_t maxp_blog(uint32_t w) {
    uint64_t b = std::min<uint64_t>((uint64_t)w + 1, kTile);
    uint32_t lg = 0;
    while ((2ull << lg) <= b) lg++;
    return lg >= 4 ? lg : 0;
}

// Slots per segment: cuts of a chain through a segment lie in
// (a, a + S + M) with spacing >= w+1; MAXP candidates lie in [a, a + S + B)
// with spacing >= w+1; both also lie inside the job's n bytes.
uint32_t slots_per_segment(uint32_t algo, uint64_t S, uint32_t w, uint32_t M,
                           uint64_t n) {
    const uint64_t span = std::min<uint64_t>(algo == kMaxp ? S + kTile : S + M, n);
    return (uint32_t)(span / ((uint64_t)w + 1) + 2);
}

uint64_t maxp_blocks(const uint8_t* data, uint64_t n, uint32_t blog) {
    if (blog == 0) return 0;
    uint64_t shift = (uintptr_t)data & 15;
    uint64_t tiles = (n + shift + kTile - 1) / kTile;
    return tiles * ((uint64_t)kTile >> blog);
}

template <class T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

struct Layout {
    size_t err, idx, succ, meta, spec, fix, rew, bmax, bpos, total;
};

// Tiles (1 KiB, address-aligned) of an n-byte buffer starting at data.
uint64_t tiles_of(const uint8_t* data, uint64_t n) {
    return (n + ((uintptr_t)data & 15) + kTile - 1) / kTile;
}

// Workspace of one job: per item a record and, for RAM / AE, the tile index
// and three cut lists (speculative, fix-up, re-walk) of `slots / items`
// entries each; for MAXP one candidate list and the block summaries.
Layout layout(uint64_t items, uint64_t slots, uint64_t blocks, bool chain,
              uint64_t tiles) {
    Layout L;
    size_t off = 0;
    L.err = off;   off += 256;
    L.idx = off;   off = align_up(off + (chain ? tiles * 16 : 0), 256);
    L.succ = off;  off = align_up(off + (chain ? tiles * 4 * kSuccSlots : 0), 256);
    L.meta = off;  off = align_up(off + items * sizeof(SegMeta), 256);
    L.spec = off;  off = align_up(off + slots * 4, 256);
    L.fix = off;   off = align_up(off + (chain ? slots * 4 : 0), 256);
    L.rew = off;   off = align_up(off + (chain ? slots * 4 : 0), 256);
    L.bpos = off;  off = align_up(off + blocks * 8, 256);
    L.bmax = off;  off = align_up(off + blocks, 256);
    L.total = off;
    return L;
}

ChainWs chain_ws(void* base, const Layout& L) {
    ChainWs w;
    w.idx = at<uint4>(base, L.idx);
    w.succ = at<uint32_t>(base, L.succ);
    w.meta = at<SegMeta>(base, L.meta);
    w.spec = at<uint32_t>(base, L.spec);
    w.fix = at<uint32_t>(base, L.fix);
    w.rew = at<uint32_t>(base, L.rew);
    w.err = at<uint32_t>(base, L.err);
    return w;
}

// Upper bounds of a batch of at most T bytes in J jobs with windows >= wmin
// and maximum chunks <= mmax: every job is split into segments of its
// algorithm's length S, and its slots per segment are bounded as in
// slots_per_segment, cap = min(S + extra, n) / (w + 1) + 2 (the chain and
// the MAXP bounds are added, since a batch may mix them).  Two bounds of
// the slots hold and the smaller is taken: per item, (T / S + J) items of
// at most A = (S + extra) / (wmin + 1) + 2 slots; and by length, a job of
// one segment holds at most n / (wmin + 1) + 2 slots, a job of several
// (n > S, so fewer than 2n / S segments) at most 2n / S * A.
BatchCaps batch_caps(uint64_t T, uint64_t J, uint64_t wmin, uint64_t mmax) {
    BatchCaps c{};
    c.seg_chain = chain_segment();
    c.seg_maxp = maxp_segment();
    c.max_chunk_limit = kMaxChunkLimit;
    const uint64_t it_chain = T / c.seg_chain + J;
    const uint64_t it_maxp = T / c.seg_maxp + J;
    c.items = std::max(it_chain, it_maxp);
    c.items_chain = it_chain;
    auto slot_bound = [&](uint64_t S, uint64_t extra) {
        const uint64_t A = (S + extra) / (wmin + 1) + 2;
        const uint64_t per_item = (T / S + J) * A;
        const uint64_t by_len = T / (wmin + 1) + 2 * J + (2 * T / S + 1) * A;
        return std::min(per_item, by_len);
    };
    c.slots = slot_bound(c.seg_chain, mmax) + slot_bound(c.seg_maxp, kTile);
    // MAXP block summaries: a job with window w uses blocks of 2^blog(w)
    // bytes, and none when blog(w) = 0 (w < 15).  Windows below 15 in the
    // batch say nothing about its MAXP jobs' windows, so the bound takes the
    // smallest block any MAXP job can use (16 bytes, blog 4) unless wmin
    // itself allows larger ones.  A job of n bytes starting at an address
    // with shift s < 16 covers ceil((n + s) / 1 KiB) <= n / 1 KiB + 2 tiles.
    const uint32_t blog = std::max<uint32_t>(
        4, maxp_blog((uint32_t)std::min<uint64_t>(wmin, 1u << 30)));
    c.blocks = (T / kTile + 2 * J + 1) * ((uint64_t)kTile >> blog);
    // tile index of the RAM / AE jobs: ceil((n + shift) / 1 KiB) per job
    c.tiles = T / kTile + 2 * J + 1;
    return c;
}

struct BatchLayout {
    size_t err, nitems, bsum, jd, items, idx, succ, meta, spec, fix, rew, bpos, bmax, total;
};

BatchLayout batch_layout(const BatchCaps& c, uint64_t n_jobs) {
    BatchLayout L;
    size_t off = 0;
    L.err = off;    off += 256;
    L.nitems = off; off += 256;
    L.bsum = off;   off = align_up(off + plan_bsum_bytes(n_jobs), 256);
    L.jd = off;     off = align_up(off + n_jobs * sizeof(JobDesc), 256);
    L.items = off;  off = align_up(off + c.items * sizeof(Item), 256);
    L.idx = off;    off = align_up(off + c.tiles * 16, 256);
    L.succ = off;   off = align_up(off + c.tiles * 4 * kSuccSlots, 256);
    L.meta = off;   off = align_up(off + c.items * sizeof(SegMeta), 256);
    L.spec = off;   off = align_up(off + c.slots * 4, 256);
    L.fix = off;    off = align_up(off + c.slots * 4, 256);
    L.rew = off;    off = align_up(off + c.slots * 4, 256);
    L.bpos = off;   off = align_up(off + c.blocks * 8, 256);
    L.bmax = off;   off = align_up(off + c.blocks, 256);
    L.total = off;
    return L;
}

// Bytes a single-buffer call needs.
size_t single_need(uint32_t algo, uint64_t n, uint32_t w, uint32_t M,
                   uint64_t shift) {
    const uint64_t S = choose_segment(algo, n);
    const uint64_t nseg = (n + S - 1) / S;
    const uint64_t cap = slots_per_segment(algo, S, w, M, n);
    const uint32_t blog = algo == kMaxp ? maxp_blog(w) : 0;
    const uint64_t blocks =
        blog ? (n + shift + kTile - 1) / kTile * ((uint64_t)kTile >> blog) : 0;
    return layout(nseg, nseg * cap, blocks, algo != kMaxp,
                  (n + shift + kTile - 1) / kTile).total;
}

// Largest grid (in waves) the per-item kernels are launched with; they walk
// the items grid-stride.
constexpr uint64_t kMaxGridWaves = 16384;

// The plan of a single-buffer call: validation, its one job and its
// workspace layout.  wpb receives the waves per workgroup in effect.
int plan_one(cdc_algo algo, const cdc_params* p, const uint8_t* data, size_t n,
             uint64_t* cut_offsets, uint64_t* n_cuts, JobDesc& jd, Layout& L,
             int& wpb) {
    if (!p || !n_cuts || (n > 0 && (!data || !cut_offsets)) ||
        p->flags != 0 || p->reserved != 0 ||
        !params_valid((uint32_t)algo, p->window, p->max_chunk)) {
        t_last_error = "invalid argument";
        return CDC_EINVAL;
    }
    if (n == 0) return CDC_OK;
    jd.data = data;
    jd.n = n;
    jd.cuts = cut_offsets;
    jd.n_cuts = n_cuts;
    jd.status = nullptr;
    jd.algo = (uint32_t)algo;
    jd.w = p->window;
    jd.M = p->max_chunk;
    {
        std::lock_guard<std::mutex> g(g_mu);
        jd.seg = choose_segment(jd.algo, n);
        wpb = g_waves_per_block;
    }
    jd.nseg = (uint32_t)((n + jd.seg - 1) / jd.seg);
    jd.item0 = 0;
    jd.cap = slots_per_segment(jd.algo, jd.seg, jd.w, jd.M, n);
    jd.slot0 = 0;
    jd.blk0 = 0;
    jd.idx0 = 0;
    jd.blog = jd.algo == kMaxp ? maxp_blog(jd.w) : 0;
    jd.ok = 1;
    const uint64_t slots = (uint64_t)jd.nseg * jd.cap;
    const uint64_t blocks = jd.algo == kMaxp ? maxp_blocks(data, n, jd.blog) : 0;
    L = layout(jd.nseg, slots, blocks, jd.algo != kMaxp, tiles_of(data, n));
    return CDC_OK;
}

// n == 0: no offsets, a count of zero.
int set_empty(uint64_t* n_cuts, hipStream_t st) {
    hipError_t e = launch_set_u64(n_cuts, 0, st);
    if (e != hipSuccess) { set_error("launch", e); return CDC_EHIP; }
    return CDC_OK;
}

// Enqueue the passes of one planned job over the workspace at `base`
// (device memory laid out as L).
int enqueue_one(const JobDesc& jd, const Layout& L, void* base, int wpb,
                hipStream_t stream, Marks* mk) {
    Plan P{};
    P.jobs = nullptr;
    P.one = jd;
    P.one_items = jd.nseg;
    hipError_t e;
    if (jd.algo == kMaxp) {
        e = launch_maxp(P, jd.nseg, 1, nullptr, at<SegMeta>(base, L.meta),
                        at<uint32_t>(base, L.spec), at<uint8_t>(base, L.bmax),
                        at<int64_t>(base, L.bpos), at<uint32_t>(base, L.err),
                        wpb, jd.blog != 0, stream, mk);
    } else {
        e = launch_ram_ae(P, jd.nseg, 1, nullptr, chain_ws(base, L), wpb,
                          stream, mk,
                          jd.nseg >= kGateMinSeg ? kPartAll : kPartAll & ~kPartGates);
    }
    if (e != hipSuccess) { set_error("kernel launch", e); return CDC_EHIP; }
    return CDC_OK;
}

// Scratch of the entry point that allocates nothing (cdc_chunk_noalloc):
// one fixed array per device, in the code object, zero at load.  In host
// code `scratch` names a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device, with that device current, and only
// that address is ever passed to kernels.  Its first word collects the
// kernels' sticky error flags (cleared by cdc_check_device_errors).
constexpr size_t kScratchBytes = 64u << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's scratch address (looked up on its first use).
int scratch_base(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_error("hipGetDevice", e); return CDC_EHIP; }
    if (dev < 0 || dev >= kMaxDevices) {
        t_last_error = "cdc_chunk_noalloc: device index out of range";
        return CDC_ENOTSUP;
    }
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("hipGetSymbolAddress(scratch)", e);
            return CDC_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CDC_OK;
}

}  // namespace

void drop_workspace(hipStream_t st) {
    std::lock_guard<std::mutex> g(g_mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto it = g_ws.find({dev, (uintptr_t)st});
    if (it == g_ws.end()) return;
    if (it->second.dev) (void)hipFree(it->second.dev);
    for (void* r : it->second.retired) (void)hipFree(r);
    it->second.side.destroy();
    for (auto& r : it->second.marks.recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : it->second.marks.pool) (void)hipEventDestroy(e);
    g_ws.erase(it);
}

}  // namespace cdc

using namespace cdc;

extern "C" {

size_t cdc_max_cuts(const cdc_params* p, size_t n) {
    if (!p || p->window == 0) return 0;
    return n == 0 ? 0 : (n - 1) / ((size_t)p->window + 1) + 1;
}

const char* cdc_status_string(int status) {
    switch (status) {
        case CDC_OK: return "ok";
        case CDC_EINVAL: return "invalid argument";
        case CDC_ENOMEM: return "workspace too small";
        case CDC_EHIP: return "HIP error";
        case CDC_ENOTSUP: return "not supported";
    }
    return "unknown status";
}

const char* cdc_last_error(void) { return t_last_error.c_str(); }

int cdc_set_tuning(const cdc_tuning* t) {
    const cdc_tuning z{0, 0, 0, 0};
    if (!t) t = &z;
    auto bad_seg = [](uint64_t s) { return s != 0 && (s < 16 || s > kMaxSeg); };
    if (bad_seg(t->chain_segment) || bad_seg(t->maxp_segment)) return CDC_EINVAL;
    if (t->waves_per_block > 4) return CDC_EINVAL;   // kernels are built for <= 256 threads
    if (t->reserved != 0) return CDC_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    g_chain_segment = t->chain_segment;
    g_maxp_segment = t->maxp_segment;
    g_waves_per_block = t->waves_per_block ? (int)t->waves_per_block : 4;
    return CDC_OK;
}

int cdc_get_tuning(cdc_tuning* t) {
    if (!t) return CDC_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    t->chain_segment = chain_segment();
    t->maxp_segment = maxp_segment();
    t->waves_per_block = (uint32_t)g_waves_per_block;
    t->reserved = 0;
    return CDC_OK;
}

int cdc_chunk(cdc_algo algo, const cdc_params* p, const uint8_t* data,
              size_t n, uint64_t* cut_offsets, uint64_t* n_cuts,
              hipStream_t stream) {
    t_last_error.clear();
    JobDesc jd{};
    Layout L{};
    int wpb = 0;
    int rc = plan_one(algo, p, data, n, cut_offsets, n_cuts, jd, L, wpb);
    if (rc != CDC_OK || n == 0) return rc == CDC_OK ? set_empty(n_cuts, stream) : rc;
    std::lock_guard<std::mutex> g(g_mu);
    Workspace& ws = workspace_for(stream);
    rc = ensure(ws, L.total, stream);
    if (rc != CDC_OK) return rc;
    ws.marks.level = g_profile_level;
    Marks* mk = g_profile_level > 0 ? &ws.marks : nullptr;
    ws.last_items = jd.algo == kMaxp ? 0u : jd.nseg;
    ws.last_meta = L.meta;
    return enqueue_one(jd, L, ws.dev, wpb, stream, mk);
}

int cdc_chunk_noalloc(cdc_algo algo, const cdc_params* p, const uint8_t* data,
                      size_t n, uint64_t* cut_offsets, uint64_t* n_cuts,
                      hipStream_t stream) {
    t_last_error.clear();
    JobDesc jd{};
    Layout L{};
    int wpb = 0;
    int rc = plan_one(algo, p, data, n, cut_offsets, n_cuts, jd, L, wpb);
    if (rc != CDC_OK || n == 0) return rc == CDC_OK ? set_empty(n_cuts, stream) : rc;
    if (L.total > kScratchBytes) {
        char buf[160];
        snprintf(buf, sizeof buf,
                 "cdc_chunk_noalloc: this call needs %zu bytes of scratch, more "
                 "than the %zu the entry point has", L.total, kScratchBytes);
        t_last_error = buf;
        return CDC_ENOMEM;
    }
    void* base = nullptr;
    rc = scratch_base(&base);
    if (rc != CDC_OK) return rc;
    return enqueue_one(jd, L, base, wpb, stream, nullptr);
}

int cdc_reserve(hipStream_t stream, size_t max_total_bytes, uint32_t max_jobs,
                uint32_t min_window, uint32_t max_chunk) {
    t_last_error.clear();
    if (min_window == 0 || max_jobs == 0 || max_chunk < min_window + 1ull ||
        max_chunk > kMaxChunkLimit)
        return CDC_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    Workspace& ws = workspace_for(stream);
    const BatchCaps caps =
        batch_caps(max_total_bytes, max_jobs, min_window, max_chunk);
    size_t need = batch_layout(caps, max_jobs).total;
    for (uint32_t algo = 0; algo < 4; algo++)
        need = std::max(need, single_need(algo, max_total_bytes, min_window,
                                          max_chunk, 15));
    const int rc = ensure(ws, need, stream);
    if (rc != CDC_OK) return rc;
    ws.res_jobs = max_jobs;
    ws.res_caps = caps;
    return CDC_OK;
}

void cdc_release(void) {
    std::lock_guard<std::mutex> g(g_mu);
    for (auto& kv : g_ws) {
        if (kv.second.dev || !kv.second.retired.empty()) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(kv.first.first);
            if (kv.second.dev) (void)hipFree(kv.second.dev);
            for (void* r : kv.second.retired) (void)hipFree(r);
            kv.second.side.destroy();
            (void)hipSetDevice(cur);
        }
    }
    g_ws.clear();
}

int cdc_chunk_batch(const cdc_job* jobs, uint32_t n_jobs, hipStream_t stream) {
    return cdc::batch_run(jobs, n_jobs, 0, true, stream);
}

}  // extern "C"

// A batch whose total length the caller knows (bytes_hint > 0) launches its
// kernels with grids sized for that length; the kernels walk the planned
// items grid-stride, so the grid only sets how many workgroups share them.
// With side = false the algorithms run in order on `stream` (for callers
// that overlap batches on streams of their own).
int cdc::batch_run(const cdc_job* jobs, uint32_t n_jobs, uint64_t bytes_hint,
                   bool side, hipStream_t stream, uint32_t algo_mask,
                   uint64_t ram_max_n) {
    t_last_error.clear();
    if (!jobs || n_jobs == 0) {
        t_last_error = "invalid argument";
        return CDC_EINVAL;
    }
    std::unique_lock<std::mutex> g(g_mu);
    return batch_on(workspace_for(stream), jobs, n_jobs, bytes_hint, side, stream,
                    algo_mask, ram_max_n);
}

// The batch on workspace `ws` (g_mu held).  Jobs of algorithms outside
// algo_mask must not occur (their passes are not enqueued).
int cdc::batch_on(Workspace& ws, const cdc_job* jobs, uint32_t n_jobs,
                  uint64_t bytes_hint, bool side, hipStream_t stream,
                  uint32_t algo_mask, uint64_t ram_max_n) {
    BatchCaps caps = ws.res_caps;
    if (ws.res_jobs < n_jobs) {
        // No reservation covers this batch: read the descriptors back to size
        // the workspace (not possible while the stream is being captured).
        if (capturing(stream)) {
            t_last_error = "batch needs cdc_reserve before stream capture";
            return CDC_ENOMEM;
        }
        std::vector<cdc_job> h(n_jobs);
        hipError_t e = hipMemcpyAsync(h.data(), jobs, n_jobs * sizeof(cdc_job),
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) { set_error("reading job descriptors", e); return CDC_EHIP; }
        uint64_t T = 0, wmin = ~0ull, mmax = 1;
        for (const cdc_job& q : h) {
            T += q.n;
            if (q.window >= 1) wmin = std::min<uint64_t>(wmin, q.window);
            mmax = std::max<uint64_t>(mmax, std::min<uint64_t>(q.max_chunk, kMaxChunkLimit));
        }
        if (wmin == ~0ull) wmin = 1;
        caps = batch_caps(T, n_jobs, wmin, mmax);
        const int rc = ensure(ws, batch_layout(caps, n_jobs).total, stream);
        if (rc != CDC_OK) return rc;
    }
    const BatchLayout L = batch_layout(caps, n_jobs);
    if (L.total > ws.cap) {
        t_last_error = "batch does not fit the reserved workspace";
        return CDC_ENOMEM;
    }
    JobDesc* jd = at<JobDesc>(ws.dev, L.jd);
    Item* items = at<Item>(ws.dev, L.items);
    uint32_t* nitems = at<uint32_t>(ws.dev, L.nitems);
    hipError_t e = launch_plan(const_cast<cdc_job*>(jobs), n_jobs, caps, jd,
                               items, nitems, at<uint8_t>(ws.dev, L.bsum), stream);
    if (e != hipSuccess) { set_error("plan launch", e); return CDC_EHIP; }
    Plan P{};
    P.jobs = jd;
    P.items = items;
    P.n_items = nitems;
    uint64_t items_upper = caps.items;
    if (bytes_hint > 0)
        items_upper = std::min<uint64_t>(
            items_upper, batch_caps(bytes_hint, n_jobs, 1, 2).items);
    const uint32_t grid_waves = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(items_upper, kMaxGridWaves));
    ws.marks.level = g_profile_level;
    Marks* mk = g_profile_level > 0 ? &ws.marks : nullptr;
    ChainWs cw;
    cw.idx = at<uint4>(ws.dev, L.idx);
    cw.succ = at<uint32_t>(ws.dev, L.succ);
    cw.meta = at<SegMeta>(ws.dev, L.meta);
    cw.spec = at<uint32_t>(ws.dev, L.spec);
    cw.fix = at<uint32_t>(ws.dev, L.fix);
    cw.rew = at<uint32_t>(ws.dev, L.rew);
    cw.err = at<uint32_t>(ws.dev, L.err);
    const int wpb = g_waves_per_block;
    // the algorithms of a batch are independent: side by side on their own
    // streams (created on first use outside capture; until then in order)
    SideStreams& sd = ws.side;
    if (side && !sd.ok && !capturing(stream) && !sd.create()) sd.destroy();
    auto maxp = [&](hipStream_t st) {
        return launch_maxp(P, grid_waves, n_jobs, nullptr, cw.meta, cw.spec,
                           at<uint8_t>(ws.dev, L.bmax), at<int64_t>(ws.dev, L.bpos),
                           cw.err, wpb, caps.blocks != 0, st, mk);
    };
    // the gate pass only where a RAM job can reach kGateMinSeg segments
    const int no_gates = ram_max_n > (kGateMinSeg - 1) * caps.seg_chain ? 0 : kPartGates;
    const uint64_t chain_items =
        bytes_hint > 0 ? std::min(caps.items_chain,
                                  batch_caps(bytes_hint, n_jobs, 1, 2).items_chain)
                       : caps.items_chain;
    const bool ae_succ = chain_items <= kAeSuccItems;
    auto chain = [&](uint32_t algo, hipStream_t st, int part) {
        return launch_chain(P, algo, grid_waves, n_jobs, nullptr, cw, st, mk,
                            part & ~no_gates, ae_succ);
    };
    const bool has_ram = algo_mask & (1u << kRam), has_ae = algo_mask & (1u << kAe);
    const bool has_min = algo_mask & (1u << kAeMin), has_maxp = algo_mask & (1u << kMaxp);
    if (side && sd.ok) {
        // The streaming passes are enqueued first, so that the host's
        // enqueueing does not hold back their start.
        e = hipEventRecord(sd.fork, stream);
        for (int i = 0; i < kSide && e == hipSuccess; i++)
            e = hipStreamWaitEvent(sd.s[i], sd.fork, 0);
        // (running RAM's index pass alone first, with the other streaming
        // passes beside RAM's walkers, made the three-job step and a
        // 6,000-job batch slower: 0.856 against 0.842 ms, 0.892 against 0.834)
        if (e == hipSuccess && has_ram) e = chain(kRam, stream, kPartIndex | kPartSpec);
        if (e == hipSuccess && has_ae) e = chain(kAe, sd.s[0], kPartIndex | kPartSpec);
        if (e == hipSuccess && has_maxp) e = maxp(sd.s[1]);
        if (e == hipSuccess && has_ram)
            e = chain(kRam, stream, kPartFix | kPartRest | kPartGates);
        if (e == hipSuccess && has_ae) e = chain(kAe, sd.s[0], kPartFix | kPartRest);
        if (e == hipSuccess && has_min) e = chain(kAeMin, sd.s[0], kPartAll);
        // the side streams join back even after a failed launch, so that no
        // side work outlives the caller's stream order
        for (int i = 0; i < kSide; i++) {
            hipError_t j = hipEventRecord(sd.join[i], sd.s[i]);
            if (j == hipSuccess) j = hipStreamWaitEvent(stream, sd.join[i], 0);
            if (e == hipSuccess) e = j;
        }
        if (e == hipSuccess && (has_ram || has_ae || has_min))
            e = launch_emit(P, grid_waves, cw, wpb, stream, mk);
    } else {
        for (uint32_t a : {kRam, kAe, kAeMin})
            if (e == hipSuccess && (algo_mask & (1u << a))) e = chain(a, stream, kPartAll);
        if (e == hipSuccess && (has_ram || has_ae || has_min))
            e = launch_emit(P, grid_waves, cw, wpb, stream, mk);
        if (e == hipSuccess && has_maxp) e = maxp(stream);
    }
    if (e != hipSuccess) { set_error("kernel launch", e); return CDC_EHIP; }
    return CDC_OK;
}

extern "C" {

int cdc_chunk_each(cdc_job* host_jobs, uint32_t n_jobs, hipStream_t stream) {
    if (!host_jobs) return CDC_EINVAL;
    int first_error = CDC_OK;
    for (uint32_t j = 0; j < n_jobs; j++) {
        cdc_job& q = host_jobs[j];
        const cdc_params p{q.window, q.max_chunk, 0, 0};
        const int rc = cdc_chunk((cdc_algo)q.algo, &p, q.data, q.n,
                                 q.cut_offsets, q.n_cuts, stream);
        q.status = rc;
        if (rc == CDC_EHIP) return rc;
        if (rc != CDC_OK && first_error == CDC_OK) first_error = rc;
    }
    return first_error;
}

int cdc_set_profiling(int level) {
    if (level < 0 || level > 2) return CDC_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    g_profile_level = level;
    return CDC_OK;
}

int cdc_kernel_times(hipStream_t stream, const char** names, uint32_t* calls,
                     double* total_ms, int max_kernels) {
    std::lock_guard<std::mutex> g(g_mu);
    Workspace& ws = workspace_for(stream);
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) { set_error("hipStreamSynchronize", e); return CDC_EHIP; }
    int used = 0;
    for (auto& r : ws.marks.recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0.f;
        int i = 0;
        while (i < used && strcmp(names[i], r.name) != 0) i++;
        if (i == used) {
            if (used == max_kernels) continue;
            names[used] = r.name;
            calls[used] = 0;
            total_ms[used] = 0.0;
            used++;
        }
        calls[i]++;
        total_ms[i] += ms;
    }
    for (auto& r : ws.marks.recs) {
        ws.marks.pool.push_back(r.a);
        ws.marks.pool.push_back(r.b);
    }
    ws.marks.recs.clear();
    return used;
}

int cdc_walk_stats(hipStream_t stream, cdc_walk_stats_t* out) {
    if (out == nullptr) return CDC_EINVAL;
    std::lock_guard<std::mutex> g(g_mu);
    Workspace& ws = workspace_for(stream);
    *out = cdc_walk_stats_t{};
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) { set_error("hipStreamSynchronize", e); return CDC_EHIP; }
    if (ws.last_items == 0 || ws.dev == nullptr) return CDC_OK;
    std::vector<SegMeta> m(ws.last_items);
    e = hipMemcpy(m.data(), static_cast<char*>(ws.dev) + ws.last_meta,
                  m.size() * sizeof(SegMeta), hipMemcpyDeviceToHost);
    if (e != hipSuccess) { set_error("hipMemcpy", e); return CDC_EHIP; }
    out->segments = m.size();
    for (const SegMeta& r : m) {
        out->steps_successor += r.steps[0];
        out->steps_fast += r.steps[1];
        out->steps_run += r.steps[2];
        out->steps_exact += r.steps[3];
        out->tiles_read_ebs += r.reads & 0xFFFFu;
        out->tiles_read_rs += r.reads >> 16;
    }
    return CDC_OK;
}

int cdc_check_device_errors(hipStream_t stream) {
    std::lock_guard<std::mutex> g(g_mu);
    Workspace& ws = workspace_for(stream);
    int dev = 0;
    (void)hipGetDevice(&dev);
    void* words[2] = {ws.dev, dev >= 0 && dev < kMaxDevices ? g_scratch_ptr[dev] : nullptr};
    uint32_t flags = 0;
    for (void* w : words) {
        if (!w) continue;
        uint32_t f = 0;
        hipError_t e = hipMemcpyAsync(&f, w, 4, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) e = hipMemsetAsync(w, 0, 4, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) { set_error("error word", e); return CDC_EHIP; }
        flags |= f;
    }
    return (int)flags;
}

}  // extern "C"

// ------------------------------------------------------------ streams

// A stream chunked in pieces (include/cdc.h, cdc_stream_*): its device
// state and buffers, and a workspace of its own, reserved at open for
// batches of one job up to the larger of the largest piece and the staged
// tail + piece head, so that its batch calls never read descriptors back.
struct cdc_stream {
    cdc::StreamDev dev{};
    void* mem = nullptr;
    cdc::Workspace ws;
    uint64_t max_piece = 0;
    uint64_t staged = 0;       // tail capacity: max_chunk + w + 64
    hipStream_t stream = nullptr;
    int device = 0;
    bool finished = false;
};

namespace {

uint64_t stream_room(uint64_t len, uint64_t w, uint64_t M) {
    return (len + 2 * M + 2 * w + 128) / (w + 1) + 4;
}

}  // namespace

extern "C" {

int cdc_stream_open(cdc_algo algo, const cdc_params* p, size_t max_piece,
                    hipStream_t stream, cdc_stream** out) {
    t_last_error.clear();
    if (!out || !p || p->flags != 0 || p->reserved != 0 || max_piece == 0 ||
        !params_valid((uint32_t)algo, p->window, p->max_chunk)) {
        t_last_error = "invalid argument";
        return CDC_EINVAL;
    }
    *out = nullptr;
    cdc_stream* S = new (std::nothrow) cdc_stream;
    if (!S) return CDC_ENOMEM;
    const uint64_t w = p->window, M = p->max_chunk;
    S->staged = M + w + 64;
    S->max_piece = max_piece;
    S->stream = stream;
    (void)hipGetDevice(&S->device);
    const uint64_t stage_cap = (2 * S->staged) / (w + 1) + 4;
    // state | tail | joined | stage | job
    const size_t o_tail = 256, o_join = align_up(o_tail + S->staged, 256),
                 o_stage = align_up(o_join + 2 * S->staged, 256),
                 o_job = align_up(o_stage + 8 * stage_cap, 256),
                 total = align_up(o_job + sizeof(cdc_job), 256);
    if (hipMalloc(&S->mem, total) != hipSuccess) {
        delete S;
        t_last_error = "hipMalloc of stream buffers failed";
        return CDC_ENOMEM;
    }
    char* b = static_cast<char*>(S->mem);
    cdc::StreamDev& D = S->dev;
    D.st = reinterpret_cast<cdc::StreamState*>(b);
    D.tail = reinterpret_cast<uint8_t*>(b + o_tail);
    D.joined = reinterpret_cast<uint8_t*>(b + o_join);
    D.stage = reinterpret_cast<uint64_t*>(b + o_stage);
    D.stage_cap = stage_cap;
    D.job = reinterpret_cast<cdc_job*>(b + o_job);
    D.tail_cap = S->staged;
    D.algo = (uint32_t)algo;
    D.w = p->window;
    D.M = p->max_chunk;
    D.lambda = algo == CDC_MAXP ? p->window : 1u;
    int rc = CDC_OK;
    {
        std::lock_guard<std::mutex> g(g_mu);
        const uint64_t T = std::max<uint64_t>(max_piece, 2 * S->staged);
        const BatchCaps caps = batch_caps(T, 1, w, M);
        rc = ensure(S->ws, batch_layout(caps, 1).total, stream);
        if (rc == CDC_OK) {
            S->ws.res_jobs = 1;
            S->ws.res_caps = caps;
        }
    }
    if (rc == CDC_OK && cdc::launch_stream_reset(D, stream) != hipSuccess) rc = CDC_EHIP;
    if (rc != CDC_OK) {
        cdc_stream_close(S);
        return rc;
    }
    *out = S;
    return CDC_OK;
}

size_t cdc_stream_max_cuts(const cdc_stream* s, size_t len) {
    if (!s) return 0;
    return (size_t)stream_room(len, s->dev.w, s->dev.M);
}

int cdc_stream_push(cdc_stream* s, const uint8_t* piece, size_t len, int last,
                    uint64_t* cut_offsets, uint64_t* n_cuts, hipStream_t stream) {
    t_last_error.clear();
    if (!s || !n_cuts || !cut_offsets || (len > 0 && !piece) ||
        len > s->max_piece || stream != s->stream || s->finished) {
        t_last_error = !s ? "invalid argument"
                     : s->finished ? "the stream has ended (cdc_stream_reset starts a new one)"
                     : stream != s->stream ? "pushes must use the stream the stream object was opened on"
                     : "invalid argument";
        return CDC_EINVAL;
    }
    const cdc::StreamDev& D = s->dev;
    if (len == 0 && !last) return set_empty(n_cuts, stream);
    const uint64_t jp = std::min<uint64_t>(len, s->staged);
    std::lock_guard<std::mutex> g(g_mu);
    hipError_t e = cdc::launch_stream_join(D, piece, jp, stream);
    if (e != hipSuccess) { set_error("stream launch", e); return CDC_EHIP; }
    const uint32_t mask = 1u << D.algo;
    int rc = batch_on(s->ws, D.job, 1, 2 * s->staged, false, stream, mask);
    if (rc != CDC_OK) return rc;
    e = cdc::launch_stream_mid(D, piece, len, jp, last ? 1 : 0, cut_offsets, stream);
    if (e != hipSuccess) { set_error("stream launch", e); return CDC_EHIP; }
    if (jp < len) {
        rc = batch_on(s->ws, D.job, 1, len, false, stream, mask);
        if (rc != CDC_OK) return rc;
    }
    e = cdc::launch_stream_fin(D, piece, len, jp, last ? 1 : 0, cut_offsets, n_cuts,
                               stream);
    if (e != hipSuccess) { set_error("stream launch", e); return CDC_EHIP; }
    if (last) s->finished = true;
    return CDC_OK;
}

int cdc_stream_reset(cdc_stream* s, hipStream_t stream) {
    if (!s || stream != s->stream) return CDC_EINVAL;
    if (cdc::launch_stream_reset(s->dev, stream) != hipSuccess) return CDC_EHIP;
    s->finished = false;
    return CDC_OK;
}

void cdc_stream_close(cdc_stream* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (s->ws.dev) (void)hipFree(s->ws.dev);
        for (void* r : s->ws.retired) (void)hipFree(r);
        s->ws.side.destroy();
        for (auto& r : s->ws.marks.recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (hipEvent_t ev : s->ws.marks.pool) (void)hipEventDestroy(ev);
    }
    if (s->mem) (void)hipFree(s->mem);
    (void)hipSetDevice(cur);
    delete s;
}

}  // extern "C"
