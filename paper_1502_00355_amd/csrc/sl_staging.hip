// Copies between callers' host memory and the device through pinned
// staging buffers, the library's pool of streams, and its cache of device
// blocks.
//
// Callers hand in ordinary (pageable) host arrays.  A copy from pageable
// memory is carried out by the runtime synchronously through its own
// staging, and copies from several threads serialize there.  Here the data
// is moved chunk by chunk through two pinned buffers from a pool the library
// keeps for the life of the process: the host copy into (or out of) one
// buffer overlaps the DMA of the other, and threads use buffers of their
// own.  A buffer returned to the pool carries the event of its last DMA;
// whoever takes it next waits for that event before touching it.
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "sl_common.h"

namespace sl {

namespace {

constexpr size_t kStageBytes = size_t(16) << 20;
constexpr size_t kDirectBytes = size_t(256) << 10;   // smaller copies go straight to the runtime

struct Stage {
    unsigned char* ptr = nullptr;
    hipEvent_t ev = nullptr;
    bool pending = false;   // ev marks a DMA that may still use the buffer
};

std::mutex g_stage_mu;
std::vector<Stage*> g_stage_free[64];

sl_status acquire(int dev, Stage** out)
{
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        if (!g_stage_free[dev].empty()) {
            *out = g_stage_free[dev].back();
            g_stage_free[dev].pop_back();
            return SL_OK;
        }
    }
    auto* s = new Stage;
    if (hipHostMalloc(reinterpret_cast<void**>(&s->ptr), kStageBytes, hipHostMallocDefault) != hipSuccess) {
        delete s;
        return fail(SL_ENOMEM, "pinned staging buffer allocation failed");
    }
    if (hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(s->ptr);
        delete s;
        return fail(SL_EDEVICE, "staging event creation failed");
    }
    *out = s;
    return SL_OK;
}

void release(int dev, Stage* s)
{
    std::lock_guard<std::mutex> lk(g_stage_mu);
    g_stage_free[dev].push_back(s);
}

// The two buffers of one copy, returned to the pool on every exit path.
struct StagePair {
    int dev = -1;
    Stage* s[2] = {nullptr, nullptr};
    ~StagePair()
    {
        for (Stage* b : s)
            if (b) release(dev, b);
    }
    sl_status init()
    {
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(SL_EDEVICE, "no current device");
        sl_status r;
        if ((r = acquire(dev, &s[0])) || (r = acquire(dev, &s[1]))) return r;
        return SL_OK;
    }
};

// Waits until no DMA uses the buffer any more.
sl_status quiesce(Stage* b)
{
    if (b->pending) {
        SL_HIP(hipEventSynchronize(b->ev));
        b->pending = false;
    }
    return SL_OK;
}

}  // namespace

sl_status copy_to_device(void* dst, const void* src, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return SL_OK;
    if (bytes <= kDirectBytes) {
        SL_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
        return SL_OK;
    }
    StagePair p;
    sl_status r = p.init();
    if (r) return r;
    const auto* in = static_cast<const unsigned char*>(src);
    auto* out = static_cast<unsigned char*>(dst);
    size_t k = 0;
    for (size_t off = 0; off < bytes; off += kStageBytes, ++k) {
        Stage* b = p.s[k & 1];
        const size_t len = std::min(kStageBytes, bytes - off);
        if ((r = quiesce(b))) return r;
        std::memcpy(b->ptr, in + off, len);
        SL_HIP(hipMemcpyAsync(out + off, b->ptr, len, hipMemcpyHostToDevice, st));
        SL_HIP(hipEventRecord(b->ev, st));
        b->pending = true;
    }
    return SL_OK;
}

sl_status copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return SL_OK;
    if (bytes <= kDirectBytes) {
        SL_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
        SL_HIP(hipStreamSynchronize(st));
        return SL_OK;
    }
    StagePair p;
    sl_status r = p.init();
    if (r) return r;
    const auto* in = static_cast<const unsigned char*>(src);
    auto* out = static_cast<unsigned char*>(dst);
    const size_t chunks = (bytes + kStageBytes - 1) / kStageBytes;
    auto issue = [&](size_t c) -> sl_status {
        Stage* b = p.s[c & 1];
        const size_t off = c * kStageBytes, len = std::min(kStageBytes, bytes - off);
        sl_status rr = quiesce(b);
        if (rr) return rr;
        SL_HIP(hipMemcpyAsync(b->ptr, in + off, len, hipMemcpyDeviceToHost, st));
        SL_HIP(hipEventRecord(b->ev, st));
        b->pending = true;
        return SL_OK;
    };
    if ((r = issue(0))) return r;
    for (size_t c = 0; c < chunks; ++c) {
        if (c + 1 < chunks && (r = issue(c + 1))) return r;
        Stage* b = p.s[c & 1];
        if ((r = quiesce(b))) return r;
        const size_t off = c * kStageBytes, len = std::min(kStageBytes, bytes - off);
        std::memcpy(out + off, b->ptr, len);
    }
    return SL_OK;
}

namespace {

// One caller array and where it goes in a device image.
struct HostPart {
    size_t off;        // byte offset in the image
    const void* src;
    size_t bytes;
};

// Copies several host arrays into one device image at their offsets through
// the pinned staging buffers: each staging chunk takes the parts of the
// arrays that fall into its window of the image and goes over in one DMA.
// The bytes between the arrays (alignment padding) are left unspecified.
// Small arrays then cost no copy of their own: a mesh of ten thousand nodes
// has seven arrays of 10-260 KB, which as separate copies went through the
// runtime's own staging one after the other, across all setup threads.
sl_status copy_image_to_device(unsigned char* dst, size_t image, const HostPart* part, int n_parts,
                               hipStream_t st)
{
    if (image == 0) return SL_OK;
    StagePair p;
    sl_status r = p.init();
    if (r) return r;
    size_t k = 0;
    for (size_t w = 0; w < image; w += kStageBytes, ++k) {
        Stage* b = p.s[k & 1];
        const size_t len = std::min(kStageBytes, image - w);
        if ((r = quiesce(b))) return r;
        for (int i = 0; i < n_parts; ++i) {
            const size_t lo = std::max(w, part[i].off), hi = std::min(w + len, part[i].off + part[i].bytes);
            if (lo < hi)
                std::memcpy(b->ptr + (lo - w), static_cast<const unsigned char*>(part[i].src) + (lo - part[i].off),
                            hi - lo);
        }
        SL_HIP(hipMemcpyAsync(dst + w, b->ptr, len, hipMemcpyHostToDevice, st));
        SL_HIP(hipEventRecord(b->ev, st));
        b->pending = true;
    }
    return SL_OK;
}

}  // namespace

sl_status upload_inputs(const sl_mesh_desc& d, int64_t nnz, int64_t ninc, size_t extra, DevInputs& out,
                        hipStream_t st)
{
    const size_t n = static_cast<size_t>(d.n_nodes), t3 = 3 * static_cast<size_t>(d.n_tris);
    const size_t bytes = Arena::piece(16 * n) + 2 * Arena::piece(4 * (n + 1)) +
                         Arena::piece(4 * static_cast<size_t>(nnz)) + Arena::piece(4 * static_cast<size_t>(ninc)) +
                         Arena::piece(4 * t3) + Arena::piece(n) + extra;
    sl_status r;
    if ((r = out.ar.reserve(bytes, st))) return r;
    if ((r = out.ar.take(&out.coords, 2 * n)) || (r = out.ar.take(&out.nbr_ptr, n + 1)) ||
        (r = out.ar.take(&out.nbr_idx, static_cast<size_t>(nnz))) || (r = out.ar.take(&out.tri_ptr, n + 1)) ||
        (r = out.ar.take(&out.tri_idx, static_cast<size_t>(ninc))) || (r = out.ar.take(&out.tris, t3)) ||
        (r = out.ar.take(&out.boundary, n)))
        return r;
    // the seven pieces were carved one after the other from the arena's start
    unsigned char* const base = out.ar.base;
    auto at = [&](const void* q) { return static_cast<size_t>(static_cast<const unsigned char*>(q) - base); };
    const HostPart parts[] = {
        {at(out.coords), d.coords, 2 * n * sizeof(double)},
        {at(out.nbr_ptr), d.nbr_ptr, (n + 1) * sizeof(int32_t)},
        {at(out.nbr_idx), d.nbr_idx, static_cast<size_t>(nnz) * sizeof(int32_t)},
        {at(out.tri_ptr), d.tri_ptr, (n + 1) * sizeof(int32_t)},
        {at(out.tri_idx), d.tri_idx, static_cast<size_t>(ninc) * sizeof(int32_t)},
        {at(out.tris), d.tris, t3 * sizeof(int32_t)},
        {at(out.boundary), d.boundary, n},
    };
    return copy_image_to_device(base, out.ar.used, parts, static_cast<int>(sizeof(parts) / sizeof(parts[0])), st);
}

namespace {

std::mutex g_stream_mu;
std::vector<hipStream_t> g_stream_free[64];
std::unordered_map<hipStream_t, int> g_stream_dev;

}  // namespace

sl_status take_stream(hipStream_t* st)
{
    *st = nullptr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(SL_EDEVICE, "no current device");
    {
        std::lock_guard<std::mutex> lk(g_stream_mu);
        if (!g_stream_free[dev].empty()) {
            *st = g_stream_free[dev].back();
            g_stream_free[dev].pop_back();
            return SL_OK;
        }
    }
    hipStream_t s = nullptr;
    SL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    std::lock_guard<std::mutex> lk(g_stream_mu);
    g_stream_dev[s] = dev;
    *st = s;
    return SL_OK;
}

void give_stream(hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_stream_mu);
    auto it = g_stream_dev.find(st);
    if (it != g_stream_dev.end()) g_stream_free[it->second].push_back(st);
}

namespace {

// per device; a batch gives back a few blocks per mesh at once, and a
// free costs about 0.24 ms of host time, so the count bound is loose and
// the byte bound is what limits the cache
constexpr size_t kCacheBlocks = 4096;
constexpr size_t kCacheBytes = kBlockCacheBytes;         // per device

struct Cached {
    unsigned char* ptr;
    size_t bytes;
    hipEvent_t ev;   // recorded on the giving stream after the block's last use
};

std::mutex g_block_mu;
std::vector<Cached> g_block_cache[64];                               // oldest first
size_t g_block_cached[64];                                           // bytes held in g_block_cache
std::unordered_map<void*, std::pair<int, size_t>> g_block_info;      // every block handed out: device, bytes
std::vector<hipEvent_t> g_block_events[64];                          // events free for reuse

// Frees the oldest cached blocks of `dev` until the cache is within its
// limits (or empty), ordered on `st` after each block's last use.  The
// caller holds g_block_mu.
void trim_blocks(int dev, bool all, hipStream_t st)
{
    auto& c = g_block_cache[dev];
    while (!c.empty() && (all || c.size() > kCacheBlocks || g_block_cached[dev] > kCacheBytes)) {
        const Cached e = c.front();
        c.erase(c.begin());
        g_block_cached[dev] -= e.bytes;
        (void)hipStreamWaitEvent(st, e.ev, 0);
        (void)hipFreeAsync(e.ptr, st);
        g_block_info.erase(e.ptr);
        g_block_events[dev].push_back(e.ev);
    }
}

}  // namespace

sl_status block_take(unsigned char** p, size_t bytes, hipStream_t st)
{
    *p = nullptr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(SL_EDEVICE, "no current device");
    {
        std::lock_guard<std::mutex> lk(g_block_mu);
        auto& c = g_block_cache[dev];
        // the smallest cached block that holds `bytes` and is not much larger
        int best = -1;
        for (int k = 0; k < static_cast<int>(c.size()); ++k)
            if (c[k].bytes >= bytes && c[k].bytes <= 2 * bytes + (size_t(1) << 20) &&
                (best < 0 || c[k].bytes < c[best].bytes))
                best = k;
        if (best >= 0) {
            const Cached e = c[best];
            SL_HIP(hipStreamWaitEvent(st, e.ev, 0));
            c.erase(c.begin() + best);
            g_block_cached[dev] -= e.bytes;
            g_block_events[dev].push_back(e.ev);
            *p = e.ptr;
            return SL_OK;
        }
    }
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(p), bytes, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_block_mu);
            trim_blocks(dev, true, st);
        }
        e = hipMallocAsync(reinterpret_cast<void**>(p), bytes, st);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SL_ENOMEM, std::string("device allocation of ") + std::to_string(bytes) +
                                   " bytes failed: " + hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk(g_block_mu);
    g_block_info[*p] = {dev, bytes};
    return SL_OK;
}

void block_give(unsigned char*& p, hipStream_t st)
{
    if (!p) return;
    unsigned char* q = p;
    p = nullptr;
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_block_mu);
    const auto it = g_block_info.find(q);
    // a block of another device, or one too large to keep, is freed at once
    if (it == g_block_info.end() || it->second.first != dev || it->second.second > kCacheBytes) {
        if (it != g_block_info.end()) g_block_info.erase(it);
        (void)hipFreeAsync(q, st);
        return;
    }
    hipEvent_t ev = nullptr;
    if (!g_block_events[dev].empty()) {
        ev = g_block_events[dev].back();
        g_block_events[dev].pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        g_block_info.erase(it);
        (void)hipFreeAsync(q, st);
        return;
    }
    if (hipEventRecord(ev, st) != hipSuccess) {
        (void)hipGetLastError();
        g_block_events[dev].push_back(ev);
        g_block_info.erase(it);
        (void)hipFreeAsync(q, st);
        return;
    }
    g_block_cache[dev].push_back(Cached{q, it->second.second, ev});
    g_block_cached[dev] += it->second.second;
    trim_blocks(dev, false, st);
}

// Frees every cached block of the current device and gives the runtime's
// stream-ordered pool back its unused memory; returns once both are done.
sl_status release_cached_memory()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(SL_EDEVICE, "no current device");
    PooledStream ps;
    sl_status r = ps.init();
    if (r) return r;
    {
        std::lock_guard<std::mutex> lk(g_block_mu);
        trim_blocks(dev, true, ps.s);
    }
    SL_HIP(hipStreamSynchronize(ps.s));
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) SL_HIP(hipMemPoolTrimTo(pool, 0));
    return SL_OK;
}

}  // namespace sl
