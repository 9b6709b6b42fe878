// ptg_serve.hip -- continuous-batching tile server (a6): a persistent kernel draining a
// work-item ring in pinned host memory, and a host scheduler that admits requests by HBM
// budget, publishes their work items while earlier ones run, and completes them.  A
// submission is admitted on the submitting thread when it fits at once.
//
// Protocol (host = scheduler thread, device = persistent kernel):
//   * the request table reqs[slot] and ring items are written by the host first; then the
//     host publishes them with a release store of ctl->tail (pinned, fine-grained memory);
//   * a workgroup reserves the next item index with a fetch-add on head (device memory),
//     so reservations never retry; the index may be ahead of what is published;
//   * mirror (device memory) is the tail as last read from host memory.  The workgroup
//     holding index == mirror is the only one that reads host memory (system-scope
//     acquire of tail): when tail has moved past it, it raises mirror to tail and runs
//     its item.  Every other waiting workgroup watches mirror with a backed-off poll;
//   * a workgroup runs its item (system-scope loads of the item; unless it still holds
//     the request descriptor, the first workgroup of the request copies it from host into
//     device memory -- claimed with a compare-and-swap on desc_state[slot] -- and the
//     others read that copy once it is whole), computes the tiles with the K3 tile and
//     strip functions, then adds its tile count to done_tiles[slot] (device memory); the
//     workgroup that brings it to the request's target stores the request's sequence
//     number into done[slot] (pinned memory, system-scope release) after a system fence
//     (a request's only item skips the count and stores done[slot] directly);
//   * the host sees done[slot] == seq, completes the request, and only then reuses the
//     slot and the request's ring entries (ring space is reclaimed in ring order);
//   * parking: once the host has had nothing in flight for a while (or is shutting down)
//     it stops publishing and sets ctl->park.  The poller that sees park with tail not
//     past its index sets parked, and every workgroup whose item is unpublished leaves;
//     items below tail are all run before their holders look at park.  The host then
//     waits for the stream, and before the next launch a one-thread kernel resets head
//     and mirror to the frozen tail (abandoned reservations are all >= that tail).
// done_tiles[] only grows: each request's target is the slot's running total, so no
// device memory is cleared while the server runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ptg_general_tile.h"
#include "ptg_internal.h"
#include "ptg_strip3_tile.h"
#include "ptg_strip_tile.h"

namespace ptg {

constexpr int kReqSlots = 1024;            // requests admitted at once
constexpr size_t kServeLds = 64 * 1024;    // dynamic LDS of a serving workgroup
constexpr int kMaxTilesPerItem = 16;      // sample tiles per work item, upper bound
constexpr int64_t kParkNs = 5000000;       // nothing in flight for 5 ms: park the kernel
constexpr int64_t kSpinNs = 2000000;       // the scheduler spins until 2 ms after the last event
constexpr int64_t kStarveNs = 50000000;    // after 50 ms a waiting request blocks later ones
constexpr int64_t kQueryNs = 500000;       // stream queries of a running kernel: every 0.5 ms
constexpr int kServeWaves = 4;             // waves of a serving workgroup (256 threads)
constexpr int kMaxLatTbl = 2048;           // lattice-cache blocks one request may use (LDS table)
constexpr int64_t kLatBlockBytes = (int64_t)kLatBlkFloats * 4;
// a strip request's LDS: [StripShared | key and node work lists | one node block per wave]
constexpr int kStripSharedWords = (int)((sizeof(StripShared) + 15) / 16 * 4);
// a 3D strip request's: [Strip3Shared | basis table, key and node work lists | per-wave blocks]
constexpr int kStrip3SharedWords = (int)((sizeof(Strip3Shared) + 15) / 16 * 4);

struct ServeReqDesc {
    int32_t dim, smooth, slot;
    uint32_t seq;
    uint64_t target;  // done_tiles[slot] when this request is complete
    int64_t ntiles;
    int32_t kernel;   // PTG_TUNE_GENERAL_2D / _GENERAL_3D (tiles), PTG_TUNE_STRIP_2D (64 x 64 strips),
                      // PTG_TUNE_STRIP_3D (64 x 8 x 16 blocks)
    int32_t model;    // PTG_MODEL_GRADIENT, _ZERO_GRADIENT (2D, C1) or _HEIGHT_GRADIENT
    union {
        Fbm2dArgs a2;
        Fbm3dArgs a3;
        Fbm2dStripArgs as;
        Fbm3dStripArgs a3s;
    };
    // lattice cache (general 2D requests): 0 = the tiles hash their nodes, 1 = the tiles
    // read the cached blocks through the table, 2 = the items fill blocks (tile index t =
    // fill word t: table entry | octave << 16)
    int32_t lat_mode;
    int32_t lat_n;                // table entries
    const uint32_t *lat_host;     // pinned: [table (kMaxLatTbl words) | fill words]
    char *lat_base;               // the arena
    int64_t lat_bx0[kMaxOctaves], lat_by0[kMaxOctaves];
    int32_t lat_nbx[kMaxOctaves], lat_tbl0[kMaxOctaves];
};
static_assert(sizeof(ServeReqDesc) % 8 == 0, "descriptor is copied in 8-byte words");

struct ServeItem {
    uint32_t slot, seq;    // request slot (| kOnlyItem: the request's one item) and the
                           // sequence number of its current request
    uint32_t ntiles, tile0;
};
constexpr uint32_t kOnlyItem = 0x80000000u;
static_assert(sizeof(ServeItem) == 16, "an item is two 8-byte words");

struct ServeHostCtl {  // pinned host memory
    uint64_t tail;         // items published
    int32_t park;          // 1: workgroups whose item is not published leave
    int32_t pad;
};

struct ServeDevCtl {       // device memory
    uint64_t head;         // next item index to reserve
    uint64_t mirror;       // tail as last read from host memory (never above tail)
    uint32_t parked;       // the poller saw park with nothing left to run
    uint32_t pad;
    uint64_t done_tiles[kReqSlots];
    // device copies of the request descriptors: desc_state[slot] = seq << 2 | 1 while one
    // workgroup copies request seq's descriptor from host memory, | 2 once the copy is whole
    uint64_t desc_state[kReqSlots];
    ServeReqDesc desc[kReqSlots];
};

__global__ void k_serve_reset(ServeDevCtl *dc, uint64_t start)
{
    dc->head = start;
    dc->mirror = start;
    dc->parked = 0;
}

__device__ __forceinline__ uint64_t sys_load64(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t sys_load32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Fill one lattice-cache block (fill word t of the request): the K1 gradients of its
// kLatBlk x kLatBlk nodes, the same key and gradient functions as the tiles' own hashing.
__device__ __forceinline__ void fill_lat_block(const ServeReqDesc &rq, const uint32_t *tbl, int64_t t, int tid)
{
    const uint32_t fw = sys_load32(rq.lat_host + kMaxLatTbl + t);
    const int o = min((int)(fw >> 16), kMaxOctaves - 1);
    const int e = min((int)(fw & 0xFFFFu), rq.lat_n - 1);  // the host writes entries < lat_n
    const int nb = max(rq.lat_nbx[o], 1);
    const int local = e - rq.lat_tbl0[o];
    const int64_t bx = rq.lat_bx0[o] + local % nb, by = rq.lat_by0[o] + local / nb;
    float *dst = reinterpret_cast<float *>(rq.lat_base + (size_t)tbl[e] * 256);
    const uint32_t pre = key_prefix(rq.a2.seed, o);
    for (int q = tid; q < kLatBlk * kLatBlk; q += 256) {
        const int64_t ix = bx * kLatBlk + (q & (kLatBlk - 1)), iy = by * kLatBlk + (q >> kLatBlkLog);
        const float2 g = grad2(key_combine(absorb_index(pre, iy), key_xline(ix)));
        dst[q] = g.x;
        dst[kLatBlk * kLatBlk + q] = g.y;
    }
}

// The work of each request kind is a function of its own (not inlined into the serving
// kernel), so that each gets its own register allocation: inlined together, the 3D strip
// code's pressure made the whole kernel spill.
//
// Strips [t0, t1) of a dyadic 2D request: wave w takes t0 + w, t0 + w + 4, ... (the same
// per-strip code as the dense strip kernel, so a served strip equals that kernel's output).
template <int M, int LO, int MD>
__device__ __noinline__ void serve_strips(const Fbm2dStripArgs &a, const StripShared &sh, uint32_t *wl, int64_t t0,
                                          int64_t t1, int tid)
{
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    float2 *nodes = reinterpret_cast<float2 *>(wl + strip_shared_words(a.nodes_hashed, a.keys_total) +
                                               wave * strip_wave_words(a.nodes_total, a.keys_total, MD == 2));
    StripWave<M, float, LO, MD> w(a, sh, nodes, lane);
    for (int64_t st = t0 + wave; st < t1; st += kServeWaves) w.run(a, sh, wl, wl + a.keys_total, st);
}

template <int M, int MD>
__device__ __forceinline__ void serve_strips_lo(const Fbm2dStripArgs &a, const StripShared &sh, uint32_t *wl,
                                                int64_t t0, int64_t t1, int tid)
{
    switch (a.lo) {  // admission guarantees 1 <= lo <= 6
    case 1: serve_strips<M, 1, MD>(a, sh, wl, t0, t1, tid); break;
    case 2: serve_strips<M, 2, MD>(a, sh, wl, t0, t1, tid); break;
    case 3: serve_strips<M, 3, MD>(a, sh, wl, t0, t1, tid); break;
    case 4: serve_strips<M, 4, MD>(a, sh, wl, t0, t1, tid); break;
    case 5: serve_strips<M, 5, MD>(a, sh, wl, t0, t1, tid); break;
    default: serve_strips<M, 6, MD>(a, sh, wl, t0, t1, tid); break;
    }
}

// A strip request of any served cell model and order (admission: the zero-gradient model
// at C1 only; orders 1..3).
__device__ __forceinline__ void serve_strips_req(const Fbm2dStripArgs &a, int model, int smooth,
                                                 const StripShared &sh, uint32_t *wl, int64_t t0, int64_t t1, int tid)
{
    if (model == PTG_MODEL_ZERO_GRADIENT) {
        serve_strips_lo<1, 1>(a, sh, wl, t0, t1, tid);
    } else if (model == PTG_MODEL_HEIGHT_GRADIENT) {
        if (smooth == 1) serve_strips_lo<1, 2>(a, sh, wl, t0, t1, tid);
        else if (smooth == 2) serve_strips_lo<2, 2>(a, sh, wl, t0, t1, tid);
        else serve_strips_lo<3, 2>(a, sh, wl, t0, t1, tid);
    } else {
        if (smooth == 1) serve_strips_lo<1, 0>(a, sh, wl, t0, t1, tid);
        else if (smooth == 2) serve_strips_lo<2, 0>(a, sh, wl, t0, t1, tid);
        else serve_strips_lo<3, 0>(a, sh, wl, t0, t1, tid);
    }
}

// Blocks [t0, t1) of a dyadic 3D request, wave w taking t0 + w, t0 + w + 4, ... (the dense
// 3D strip kernel's per-block code).
template <int M, int LO, int MD>
__device__ __noinline__ void serve_blocks(const Fbm3dStripArgs &a, const Strip3Shared &sh, float4 *tab, int64_t t0,
                                          int64_t t1, int tid)
{
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int listed = a.keys_col + 4 * a.n_coarse;
    const uint32_t *wl_key = reinterpret_cast<const uint32_t *>(tab) + strip3_tab_words(a.tab_total);
    float *gx = reinterpret_cast<float *>(tab) + strip3_shared_words(a.tab_total, listed, a.nodes_listed) +
                wave * strip3_wave_words(a.nodes_total, a.keys_total, MD == 2 ? 1 : 0);
    Strip3Wave<M, float, LO, MD> w(a, sh, gx, lane);
    for (int64_t b = t0 + wave; b < t1; b += kServeWaves) w.run(a, sh, tab, wl_key, wl_key + listed, b);
}

template <int M, int MD>
__device__ __forceinline__ void serve_blocks_lo(const Fbm3dStripArgs &a, const Strip3Shared &sh, float4 *tab,
                                                int64_t t0, int64_t t1, int tid)
{
    switch (a.lo) {
    case 1: serve_blocks<M, 1, MD>(a, sh, tab, t0, t1, tid); break;
    case 2: serve_blocks<M, 2, MD>(a, sh, tab, t0, t1, tid); break;
    case 3: serve_blocks<M, 3, MD>(a, sh, tab, t0, t1, tid); break;
    default: serve_blocks<M, 4, MD>(a, sh, tab, t0, t1, tid); break;
    }
}

// General tiles [t0, t1) of a 2D / 3D request, one after the other.
template <int M, int TH, int MD>
__device__ __noinline__ void serve_tiles_2d(const Fbm2dArgs &a, const LatCache *lat, int64_t t0, int64_t t1,
                                            float4 *lds4)
{
    for (int64_t t = t0; t < t1; ++t) {
        fbm2d_general_tile<M, float, TH, MD>(a, t, lds4, lat);
        __syncthreads();  // LDS reuse by the next tile
    }
}

template <int M, int MD>
__device__ __forceinline__ void serve_tiles_2d_th(const Fbm2dArgs &a, const LatCache *lat, int64_t t0, int64_t t1,
                                                  float4 *lds4)
{
    if (a.tile_h == 16) serve_tiles_2d<M, 16, MD>(a, lat, t0, t1, lds4);
    else if (a.tile_h == 32) serve_tiles_2d<M, 32, MD>(a, lat, t0, t1, lds4);
    else serve_tiles_2d<M, 64, MD>(a, lat, t0, t1, lds4);
}

__device__ __forceinline__ void serve_tiles_2d_req(const Fbm2dArgs &a, int model, int smooth, const LatCache *lat,
                                                   int64_t t0, int64_t t1, float4 *lds4)
{
    if (model == PTG_MODEL_ZERO_GRADIENT) {
        serve_tiles_2d_th<1, 1>(a, lat, t0, t1, lds4);
    } else if (model == PTG_MODEL_HEIGHT_GRADIENT) {
        if (smooth == 1) serve_tiles_2d_th<1, 2>(a, lat, t0, t1, lds4);
        else if (smooth == 2) serve_tiles_2d_th<2, 2>(a, lat, t0, t1, lds4);
        else serve_tiles_2d_th<3, 2>(a, lat, t0, t1, lds4);
    } else {
        if (smooth == 1) serve_tiles_2d_th<1, 0>(a, lat, t0, t1, lds4);
        else if (smooth == 2) serve_tiles_2d_th<2, 0>(a, lat, t0, t1, lds4);
        else serve_tiles_2d_th<3, 0>(a, lat, t0, t1, lds4);
    }
}

template <int M, int MD>
__device__ __noinline__ void serve_tiles_3d(const Fbm3dArgs &a, int64_t t0, int64_t t1, float4 *lds4)
{
    for (int64_t t = t0; t < t1; ++t) {
        fbm3d_general_tile<M, float, MD>(a, t, lds4);
        __syncthreads();
    }
}

__device__ __forceinline__ void serve_tiles_3d_req(const Fbm3dArgs &a, int model, int smooth, int64_t t0, int64_t t1,
                                                   float4 *lds4)
{
    if (model == PTG_MODEL_HEIGHT_GRADIENT) {
        if (smooth == 1) serve_tiles_3d<1, 2>(a, t0, t1, lds4);
        else if (smooth == 2) serve_tiles_3d<2, 2>(a, t0, t1, lds4);
        else serve_tiles_3d<3, 2>(a, t0, t1, lds4);
    } else {
        if (smooth == 1) serve_tiles_3d<1, 0>(a, t0, t1, lds4);
        else if (smooth == 2) serve_tiles_3d<2, 0>(a, t0, t1, lds4);
        else serve_tiles_3d<3, 0>(a, t0, t1, lds4);
    }
}

__global__ __launch_bounds__(256, 2) void k_serve(ServeHostCtl *hc, const ServeItem *ring, const ServeReqDesc *reqs,
                                               uint32_t *done, ServeDevCtl *dc, int32_t ring_size)
{
    extern __shared__ float4 lds4[];
    __shared__ uint64_t s_req[sizeof(ServeReqDesc) / 8];
    __shared__ int s_cmd;
    __shared__ ServeItem s_item;
    __shared__ uint32_t s_have_slot, s_have_seq;  // request whose descriptor s_req holds
    __shared__ uint32_t s_tbl[kMaxLatTbl];        // its lattice-cache table
    __shared__ int s_copy;                        // 1: this workgroup copies the descriptor
    __shared__ bool s_only;                       // the item is its request's only one
    const int tid = threadIdx.x;
    if (tid == 0) s_have_slot = 0xFFFFFFFFu;
    for (;;) {
        if (tid == 0) {
            const uint64_t my = __hip_atomic_fetch_add(&dc->head, (uint64_t)1, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            int cmd = 0, nap = 8, polls = 0;
            // Polls are relaxed loads (an acquire on this chip invalidates the L2, which a
            // spinning workgroup would do continuously); one acquire fence follows success.
            for (;;) {
                const uint64_t m = __hip_atomic_load(&dc->mirror, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (my < m) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    cmd = 1;
                    break;
                }
                if (my == m) {  // first unpublished index: poll host memory (park every 8th poll)
                    const int32_t pk = (++polls & 7) != 0 ? 0
                                     : __hip_atomic_load(&hc->park, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    if (pk) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the tail read next is final
                    const uint64_t t = __hip_atomic_load(&hc->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    if (t > my) {
                        if (!pk) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                        __hip_atomic_fetch_max(&dc->mirror, t, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        cmd = 1;
                        break;
                    }
                    if (pk) {  // t == my == mirror: every published item is held below us
                        __hip_atomic_store(&dc->parked, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                } else {
                    if (__hip_atomic_load(&dc->parked, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                    for (int z = 0; z < nap; z += 8) __builtin_amdgcn_s_sleep(8);  // ~nap * 64 clocks
                    nap = nap < 128 ? 2 * nap : 128;
                }
            }
            if (cmd == 1) {
                const uint64_t *w = reinterpret_cast<const uint64_t *>(ring + (my % (uint64_t)ring_size));
                const uint64_t w0 = sys_load64(w), w1 = sys_load64(w + 1);
                s_item.slot = (uint32_t)w0 & ~kOnlyItem;
                s_only = ((uint32_t)w0 & kOnlyItem) != 0;
                s_item.seq = (uint32_t)(w0 >> 32);
                s_item.ntiles = (uint32_t)w1;
                s_item.tile0 = (uint32_t)(w1 >> 32);
                if (s_item.slot == s_have_slot && s_item.seq == s_have_seq) cmd = 2;  // descriptor held
                s_have_slot = s_item.slot;
                s_have_seq = s_item.seq;
            }
            s_cmd = cmd;
        }
        __syncthreads();
        if (s_cmd == 0) return;  // parked: every wave of the workgroup leaves
        if (s_cmd == 1) {
            // The first workgroup to run an item of the request copies its descriptor from host
            // memory into device memory; later ones (and those that arrive while it copies,
            // after waiting for it) read the device copy, so the host is read once per request.
            uint64_t *stp = &dc->desc_state[s_item.slot];
            const uint64_t want = (uint64_t)s_item.seq << 2;
            if (tid == 0 && s_only) {
                s_copy = 2;  // nobody else reads it: straight from host memory
            } else if (tid == 0) {
                uint64_t st = __hip_atomic_load(stp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                int copy = 0;
                for (;;) {
                    if (st == (want | 2)) break;
                    if (st == (want | 1)) {  // another workgroup is copying it
                        __builtin_amdgcn_s_sleep(2);
                        st = __hip_atomic_load(stp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        continue;
                    }
                    // an earlier request's state (whose items have all run): take the copy
                    if (__hip_atomic_compare_exchange_strong(stp, &st, want | 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        copy = 1;
                        break;
                    }
                }
                if (!copy) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the copy's writes
                s_copy = copy;
            }
            __syncthreads();
            const bool copy = s_copy == 1, host = s_copy != 0;
            const uint64_t *src = reinterpret_cast<const uint64_t *>(reqs + s_item.slot);
            uint64_t *dev = reinterpret_cast<uint64_t *>(dc->desc + s_item.slot);
            for (int i = tid; i < (int)(sizeof(ServeReqDesc) / 8); i += 256) {
                const uint64_t v = host ? sys_load64(src + i) : dev[i];
                s_req[i] = v;
                if (copy) dev[i] = v;
            }
            if (copy) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // each wave's copy stores
            __syncthreads();
            if (copy && tid == 0) __hip_atomic_store(stp, want | 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const ServeReqDesc &d = *reinterpret_cast<const ServeReqDesc *>(s_req);
            if (d.lat_mode != 0) {
                for (int i = tid; i < d.lat_n; i += 256) s_tbl[i] = sys_load32(d.lat_host + i);
                __syncthreads();
            }
        }
        const ServeReqDesc &rq = *reinterpret_cast<const ServeReqDesc *>(s_req);
        const int64_t t1 = (int64_t)s_item.tile0 + s_item.ntiles;
        if (rq.kernel == PTG_TUNE_STRIP_2D) {
            // the work lists stay in LDS while this workgroup's items come from one request
            StripShared &sh = *reinterpret_cast<StripShared *>(lds4);
            uint32_t *wl = reinterpret_cast<uint32_t *>(lds4) + kStripSharedWords;
            if (s_cmd == 1) {
                strip_prologue(rq.as, sh, wl, wl + rq.as.keys_total, tid, 256);
                __syncthreads();
            }
            serve_strips_req(rq.as, rq.model, rq.smooth, sh, wl, s_item.tile0, t1, tid);
            __syncthreads();
        } else if (rq.kernel == PTG_TUNE_STRIP_3D) {
            Strip3Shared &sh = *reinterpret_cast<Strip3Shared *>(lds4);
            float4 *tab = lds4 + kStrip3SharedWords / 4;
            if (s_cmd == 1) {
                uint32_t *wl_key = reinterpret_cast<uint32_t *>(tab) + strip3_tab_words(rq.a3s.tab_total);
                uint32_t *wl_node = wl_key + rq.a3s.keys_col + 4 * rq.a3s.n_coarse;
                if (rq.smooth == 1)
                    strip3_prologue<1>(rq.a3s, sh, tab, wl_key, wl_node, tid, 256);
                else
                    strip3_prologue<2>(rq.a3s, sh, tab, wl_key, wl_node, tid, 256);
                __syncthreads();
            }
            const bool hg = rq.model == PTG_MODEL_HEIGHT_GRADIENT;  // admission: orders 1, 2
            if (rq.smooth == 1) {
                if (hg) serve_blocks_lo<1, 2>(rq.a3s, sh, tab, s_item.tile0, t1, tid);
                else serve_blocks_lo<1, 0>(rq.a3s, sh, tab, s_item.tile0, t1, tid);
            } else {
                if (hg) serve_blocks_lo<2, 2>(rq.a3s, sh, tab, s_item.tile0, t1, tid);
                else serve_blocks_lo<2, 0>(rq.a3s, sh, tab, s_item.tile0, t1, tid);
            }
            __syncthreads();
        }
        if (rq.lat_mode == 2) {
            for (int64_t t = s_item.tile0; t < t1; ++t) fill_lat_block(rq, s_tbl, t, tid);
            // every wave's block stores have reached the L2 (vmcnt(0)) before the barrier, so
            // the release below writes them back: tiles of other workgroups (other XCDs) read
            // them as soon as the host has seen the fills done
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __syncthreads();
        }
        const bool tiles = rq.lat_mode != 2 && (rq.kernel == PTG_TUNE_GENERAL_2D || rq.kernel == PTG_TUNE_GENERAL_3D);
        if (tiles && rq.dim == 2) {
            const LatCache lc{rq.lat_base, s_tbl, rq.lat_n, rq.lat_bx0, rq.lat_by0, rq.lat_nbx, rq.lat_tbl0};
            const LatCache *lat = rq.lat_mode == 1 ? &lc : nullptr;
            serve_tiles_2d_req(rq.a2, rq.model, rq.smooth, lat, s_item.tile0, t1, lds4);
        } else if (tiles) {
            serve_tiles_3d_req(rq.a3, rq.model, rq.smooth, s_item.tile0, t1, lds4);
        }
        // every wave's output stores have reached the L2 before thread 0's release writes it back
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
        if (tid == 0 && s_only) {  // the request's one item: signal the host directly
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            __hip_atomic_store(done + rq.slot, rq.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        } else if (tid == 0) {
            // this workgroup's output reaches memory before it is counted (release: L2
            // write-back); only the workgroup that completes the request also acquires the
            // other workgroups' releases before it signals the host
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            const uint64_t n = (uint64_t)s_item.ntiles;
            const uint64_t old = __hip_atomic_fetch_add(&dc->done_tiles[rq.slot], n, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            if (old + n == rq.target) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(done + rq.slot, rq.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();  // s_req / s_item are rewritten by the next claim
    }
}

// ---------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------
static int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over [0, size) with 256-byte granules.
class Arena {
  public:
    explicit Arena(int64_t size) { free_[0] = size; }
    int64_t alloc(int64_t bytes)
    {
        bytes = (bytes + 255) & ~int64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest > 0) free_[off + bytes] = rest;
                used_ += bytes;
                return off;
            }
        }
        return -1;
    }
    int64_t largest_free() const
    {
        int64_t m = 0;
        for (const auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
    void release(int64_t off, int64_t bytes)
    {
        bytes = (bytes + 255) & ~int64_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t used() const { return used_; }

  private:
    int64_t used_ = 0;
    std::map<int64_t, int64_t> free_;
};

// A lattice-cache block: kLatBlk x kLatBlk nodes (bx, by) of one octave of one seed.
struct LatKey {
    uint32_t seed;
    int32_t octave;
    int64_t bx, by;
    bool operator==(const LatKey &o) const
    {
        return seed == o.seed && octave == o.octave && bx == o.bx && by == o.by;
    }
};
struct LatKeyHash {
    size_t operator()(const LatKey &k) const
    {
        uint64_t h = ((uint64_t)k.seed << 8 | (uint32_t)k.octave) * 0x9E3779B97F4A7C15ull;
        h = (h ^ (uint64_t)k.bx) * 0xBF58476D1CE4E5B9ull;
        h = (h ^ (uint64_t)k.by) * 0x94D049BB133111EBull;
        return (size_t)(h ^ (h >> 31));
    }
};
struct LatBlock {
    int64_t off = -1;
    int32_t refs = 0;        // admitted requests that use it
    uint64_t filler = 0;     // ticket whose fill phase writes it; 0 = written
    bool bad = false;        // its fill failed: dropped once unreferenced
    std::list<LatKey>::iterator lru;  // position in the LRU list while unreferenced
    std::vector<uint64_t> waiters;    // other requests that read it once written
};

struct Request {
    ptg_tile_req req;
    int64_t bytes = 0, ntiles = 0, arena_off = -1, per_item = 1, items = 0;
    int32_t kernel = 0;  // PTG_TUNE_* class that computes it
    // lattice cache: the blocks of its footprint (table order), the fill words of the ones
    // its first phase writes, and the table geometry per octave
    int32_t lat = 0, lat_n = 0;
    int64_t lat_bx0[kMaxOctaves] = {}, lat_by0[kMaxOctaves] = {};
    int32_t lat_nbx[kMaxOctaves] = {}, lat_tbl0[kMaxOctaves] = {};
    std::vector<LatKey> lat_keys;
    std::vector<uint32_t> lat_fill;
    int64_t fill_per = 1, fill_items = 0;
    int32_t next_phase = 2;  // waiting: 1 = its fills, 2 = its tiles are published next
    int32_t lat_unready = 0; // its blocks not written yet (its own fills and others')
    bool lat_bad = false;    // a block it reads will never be written (its filler failed)
    int32_t slot = -1;
    uint32_t seq = 0;
    uint64_t ring_begin = 0, ring_end = 0;
    // 1: pending, 2: tiles in flight, 3: fills in flight, 4: admitted, waiting for blocks
    // that other requests fill or for ring space; PTG_OK / error: complete
    int status = 1;
    int64_t t_submit = 0, t_admit = 0, t_done = 0, fake_done_at = 0;
};

}  // namespace ptg

struct ptg_server {
    ptg_server_cfg cfg{};
    bool gpu = true;
    int tile_h2[2] = {ptg::kTile2, ptg::kTile2};  // 2D tile height for C1 / C2 requests (C3: 64)
    hipStream_t stream = nullptr;
    int workgroups = 0;
    ptg::ServeHostCtl *hc = nullptr;
    ptg::ServeItem *ring = nullptr;
    ptg::ServeReqDesc *reqs = nullptr;
    uint32_t *done = nullptr;
    ptg::ServeDevCtl *dc = nullptr;
    char *arena_mem = nullptr;
    std::unique_ptr<ptg::Arena> arena;

    std::mutex mu;
    std::condition_variable cv_done, cv_work;
    std::deque<uint64_t> done_q;  // completed tickets in completion order (ptg_tiles_wait_any)
    std::map<uint64_t, ptg::Request> by_ticket;
    std::deque<uint64_t> pending;
    std::vector<uint64_t> inflight;
    struct RingSpan {
        uint64_t ticket, end;
        int32_t phase;  // 1: a request's fills, 2: its tiles
        bool done;
    };
    std::deque<RingSpan> ring_order;  // admitted requests in ring order
    std::vector<int32_t> free_slots;
    std::vector<uint64_t> slot_total;
    uint64_t next_ticket = 1, tail = 0, reclaimed = 0;
    uint32_t seq = 0;
    bool stopping = false, quit = false;
    bool kernel_running = false, park_requested = false;
    uint64_t base = 0;        // first item index of the next launch (tail when the last one parked)
    // lattice cache: resident blocks, the unreferenced ones in LRU order (front = oldest),
    // admitted requests waiting for their next phase, per-slot tables in pinned memory
    std::unordered_map<ptg::LatKey, ptg::LatBlock, ptg::LatKeyHash> lat_cache;
    std::list<ptg::LatKey> lat_lru;
    int64_t lat_lru_bytes = 0;
    std::vector<uint64_t> lat_waiting;
    uint32_t *lat_host = nullptr;
    int64_t idle_since = 0;   // when the in-flight set last became empty
    int64_t last_query = 0;   // last hipStreamQuery of the running kernel
    int64_t last_event = 0;   // last submission or completion
    // work units (a tile, or a workgroup's kServeWaves strips / 3D blocks) of the requests in
    // flight and of those waiting for admission: the load that sizes work items
    int64_t tiles_in_flight = 0;
    int64_t tiles_pending = 0;
    int64_t fake_busy_until = 0;
    ptg_server_stats st{};
    std::thread th;
    std::string err;
};

namespace ptg {

// Work units of a request: its tiles, or for strip requests its groups of kServeWaves strips
// (3D blocks), one per wave of a workgroup.
static int64_t work_units(int32_t kernel, int64_t ntiles)
{
    const bool strips = kernel == PTG_TUNE_STRIP_2D || kernel == PTG_TUNE_STRIP_3D;
    return strips ? (ntiles + kServeWaves - 1) / kServeWaves : ntiles;
}

// Tiles per work item: the configured count; else sized to the load.  With little in
// flight or waiting a request is cut into small items that spread over many workgroups
// (latency); with a backlog (in flight or still pending) items grow to kMaxTilesPerItem
// tiles (fewer claims and completions per tile: throughput).  Never more items than the
// ring holds (validation guarantees that kMaxTilesPerItem tiles per item fit).
static int64_t tiles_per_item(const ptg_server *s, int64_t ntiles)
{
    int64_t per = s->cfg.tiles_per_item;
    if (per <= 0) {
        const int64_t wg = std::max(s->workgroups, 1);
        const int64_t load = s->tiles_in_flight + s->tiles_pending + ntiles;
        per = std::max<int64_t>(1, std::min<int64_t>(kMaxTilesPerItem, load / (2 * wg)));
    }
    const int64_t need = (ntiles + s->cfg.max_items - 1) / s->cfg.max_items;
    return std::max(per, need);
}

static int64_t round256(int64_t b) { return (b + 255) & ~int64_t(255); }

// ---- lattice cache ------------------------------------------------------------------

// Blocks covering a 2D request's footprint per octave (every node its general tiles read):
// the table entries, or -1 beyond kMaxLatTbl.  With r, also its table geometry.
static int lat_geometry(const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny, Request *r)
{
    double freq[kMaxOctaves];
    float amp[kMaxOctaves];
    octave_tables(p, freq, amp);
    int64_t n = 0;
    for (int o = 0; o < p->octaves; ++o) {
        const double f = freq[o];
        const int64_t bx0 = cell_of(x0, f) >> kLatBlkLog, bx1 = (cell_of(x0 + nx - 1, f) + 1) >> kLatBlkLog;
        const int64_t by0 = cell_of(y0, f) >> kLatBlkLog, by1 = (cell_of(y0 + ny - 1, f) + 1) >> kLatBlkLog;
        const int64_t nbx = bx1 - bx0 + 1, nby = by1 - by0 + 1;
        if (nbx > kMaxLatTbl || nby > kMaxLatTbl || n + nbx * nby > kMaxLatTbl) return -1;
        if (r) {
            r->lat_bx0[o] = bx0;
            r->lat_by0[o] = by0;
            r->lat_nbx[o] = (int32_t)nbx;
            r->lat_tbl0[o] = (int32_t)n;
        }
        n += nbx * nby;
    }
    return (int)n;
}

static void lat_evict_oldest(ptg_server *s)
{
    const LatKey k = s->lat_lru.front();
    s->lat_lru.pop_front();
    s->lat_lru_bytes -= kLatBlockBytes;
    auto it = s->lat_cache.find(k);
    s->arena->release(it->second.off, kLatBlockBytes);
    s->lat_cache.erase(it);
    s->st.lat_evictions++;
}

// Arena bytes, evicting unreferenced lattice blocks (oldest first) when they are needed.
static int64_t arena_alloc(ptg_server *s, int64_t bytes)
{
    int64_t off = s->arena->alloc(bytes);
    if (off >= 0 || s->lat_lru.empty()) return off;
    if (s->cfg.hbm_budget_bytes - s->arena->used() + s->lat_lru_bytes < round256(bytes)) return -1;  // hopeless
    while (off < 0 && !s->lat_lru.empty()) {
        lat_evict_oldest(s);
        off = s->arena->alloc(bytes);
    }
    return off;
}

// Drop a request's references; blocks left unreferenced join the LRU list, or are freed
// when their fill never completed (failed: the request's own fills did not run).
static void lat_unref(ptg_server *s, uint64_t ticket, Request &r, bool failed)
{
    for (const LatKey &k : r.lat_keys) {
        auto it = s->lat_cache.find(k);
        LatBlock &b = it->second;
        if (failed && b.filler == ticket) {
            b.bad = true;
            for (uint64_t w : b.waiters) {
                auto wr = s->by_ticket.find(w);
                if (wr != s->by_ticket.end()) wr->second.lat_bad = true;
            }
            b.waiters.clear();
        }
        auto me = std::find(b.waiters.begin(), b.waiters.end(), ticket);
        if (me != b.waiters.end()) b.waiters.erase(me);
        if (--b.refs > 0) continue;
        if (b.bad || b.filler != 0) {
            s->arena->release(b.off, kLatBlockBytes);
            s->lat_cache.erase(it);
        } else {
            b.lru = s->lat_lru.insert(s->lat_lru.end(), k);
            s->lat_lru_bytes += kLatBlockBytes;
        }
    }
    r.lat_keys.clear();
    r.lat_fill.clear();
}

// Reference every block of a cached request; the missing ones get arena bytes and a fill
// word (its fill phase writes them).  False, holding nothing, when the arena cannot take
// the missing blocks now.
static bool lat_acquire(ptg_server *s, uint64_t ticket, Request &r)
{
    const ptg_params *p = &r.req.params;
    r.lat_n = lat_geometry(p, r.req.origin[0], r.req.origin[1], r.req.extent[0], r.req.extent[1], &r);
    r.lat_keys.clear();
    r.lat_fill.clear();
    r.lat_unready = 0;
    r.lat_bad = false;
    std::vector<uint32_t> tbl((size_t)r.lat_n);
    int64_t hits = 0;
    for (int o = 0; o < p->octaves; ++o) {
        const int nbx = r.lat_nbx[o];
        const int nby = ((o + 1 < p->octaves ? r.lat_tbl0[o + 1] : r.lat_n) - r.lat_tbl0[o]) / nbx;
        for (int j = 0; j < nby; ++j)
            for (int i = 0; i < nbx; ++i) {
                const int e = r.lat_tbl0[o] + j * nbx + i;
                const LatKey k{p->seed, o, r.lat_bx0[o] + i, r.lat_by0[o] + j};
                auto it = s->lat_cache.find(k);
                if (it == s->lat_cache.end()) {
                    const int64_t off = arena_alloc(s, kLatBlockBytes);
                    if (off < 0) {
                        lat_unref(s, ticket, r, true);
                        return false;
                    }
                    it = s->lat_cache.emplace(k, LatBlock{}).first;
                    it->second.off = off;
                    it->second.filler = ticket;
                    r.lat_fill.push_back((uint32_t)e | ((uint32_t)o << 16));
                    ++r.lat_unready;
                } else {
                    LatBlock &b = it->second;
                    if (b.refs == 0) {
                        s->lat_lru.erase(b.lru);
                        s->lat_lru_bytes -= kLatBlockBytes;
                    }
                    if (b.bad) r.lat_bad = true;
                    if (b.filler != 0 && !b.bad) {  // another request's fill writes it
                        ++r.lat_unready;
                        b.waiters.push_back(ticket);
                    }
                    ++hits;
                }
                it->second.refs++;
                r.lat_keys.push_back(k);
                tbl[(size_t)e] = (uint32_t)(it->second.off >> 8);
            }
    }
    s->st.lat_hits += hits;
    s->st.lat_misses += (int64_t)r.lat_fill.size();
    if (s->gpu) {
        uint32_t *h = s->lat_host + (size_t)r.slot * 2 * kMaxLatTbl;
        std::memcpy(h, tbl.data(), tbl.size() * 4);
        std::memcpy(h + kMaxLatTbl, r.lat_fill.data(), r.lat_fill.size() * 4);
    }
    const int64_t wg = std::max(s->workgroups, 1), nf = (int64_t)r.lat_fill.size();
    // a block is a small job (kLatBlk^2 hashes): about 8 items per request of up to 16 blocks
    // each (fewer claims and completion fences per block)
    r.fill_per = std::max<int64_t>((nf + 7) / 8, std::min<int64_t>(kMaxTilesPerItem, nf / (2 * wg)));
    r.fill_per = std::max<int64_t>(1, std::min<int64_t>(kMaxTilesPerItem, r.fill_per));
    r.fill_per = std::max<int64_t>(r.fill_per, (nf + s->cfg.max_items - 1) / s->cfg.max_items);
    r.fill_items = (nf + r.fill_per - 1) / r.fill_per;
    return true;
}

// A request's fills are done: its blocks are written, for it and for their waiters.
static void lat_filled(ptg_server *s, Request &r)
{
    for (uint32_t fw : r.lat_fill) {
        LatBlock &b = s->lat_cache.find(r.lat_keys[fw & 0xFFFFu])->second;
        b.filler = 0;
        --r.lat_unready;
        for (uint64_t w : b.waiters) {
            auto wr = s->by_ticket.find(w);
            if (wr != s->by_ticket.end()) --wr->second.lat_unready;
        }
        b.waiters.clear();
    }
}

// ---- request life cycle ---------------------------------------------------------------

// Ring entries are reused in ring order: mark a published span finished and reclaim up to
// the first unfinished one.
static void span_done(ptg_server *s, uint64_t ticket, int32_t phase)
{
    for (auto &e : s->ring_order)
        if (e.ticket == ticket && (phase == 0 || e.phase == phase)) e.done = true;
    while (!s->ring_order.empty() && s->ring_order.front().done) {
        s->reclaimed = s->ring_order.front().end;
        s->ring_order.pop_front();
    }
}

static void complete(ptg_server *s, uint64_t ticket, int status)
{
    Request &r = s->by_ticket[ticket];
    if (r.status == 2) s->tiles_in_flight -= work_units(r.kernel, r.ntiles);
    if (r.lat) lat_unref(s, ticket, r, status != PTG_OK);
    r.status = status;
    r.t_done = now_ns();
    s->last_event = r.t_done;
    if (r.slot >= 0) s->free_slots.push_back(r.slot);
    span_done(s, ticket, 0);
    s->st.completed++;
    if (status == PTG_OK) s->st.tiles_done += r.ntiles;
    s->st.bytes_in_use = s->arena->used();
    s->done_q.push_back(ticket);
    s->cv_done.notify_all();
}

// 2D general-tile height of a served request: the configured or tuned one for C1 / C2, 64
// rows for higher orders.
static int served_tile_h(const ptg_server *s, int smooth) { return smooth <= 2 ? s->tile_h2[smooth - 1] : kTile2; }

// Publish one phase of an admitted request (slot held): 1 = the fills of its missing
// lattice blocks, 2 = its tiles.
static void publish(ptg_server *s, uint64_t ticket, Request &r, int phase)
{
    const int32_t slot = r.slot;
    r.seq = ++s->seq;
    r.status = phase == 1 ? 3 : 2;
    const int64_t nwork = phase == 1 ? (int64_t)r.lat_fill.size() : r.ntiles;
    const int64_t per = phase == 1 ? r.fill_per : r.per_item;
    const uint64_t items = (uint64_t)(phase == 1 ? r.fill_items : r.items);
    if (phase == 2) s->tiles_in_flight += work_units(r.kernel, r.ntiles);
    r.ring_begin = s->tail;
    r.ring_end = s->tail + items;
    s->ring_order.push_back({ticket, r.ring_end, phase, false});
    s->inflight.push_back(ticket);
    s->st.bytes_in_use = s->arena->used();
    s->st.bytes_peak = std::max(s->st.bytes_peak, s->st.bytes_in_use);
    if (!s->gpu) {
        s->fake_busy_until = std::max(s->fake_busy_until, now_ns()) + nwork * s->cfg.fake_tile_ns;
        r.fake_done_at = s->fake_busy_until;
        s->tail = r.ring_end;
        return;
    }
    ServeReqDesc d;
    std::memset(&d, 0, sizeof(d));
    const ptg_params *p = &r.req.params;
    void *out = s->arena_mem + r.arena_off;
    d.dim = p->dim;
    d.smooth = p->smoothness;
    d.slot = slot;
    d.seq = r.seq;
    // a request's one item signals the host itself; done_tiles[slot] counts the others' tiles
    if (items > 1) s->slot_total[slot] += (uint64_t)nwork;
    d.target = s->slot_total[slot];
    d.ntiles = nwork;
    d.kernel = r.kernel;
    d.model = p->model;
    if (r.kernel == PTG_TUNE_STRIP_2D) {
        int k = 0;
        (void)dyadic_shift(p, &k);  // validated at submission
        (void)strip_args_2d(p, k, r.req.origin[0], r.req.origin[1], r.req.extent[0], r.req.extent[1], out,
                            r.req.extent[0], &d.as);
    } else if (r.kernel == PTG_TUNE_STRIP_3D) {
        int k = 0;
        (void)dyadic_shift(p, &k);
        (void)strip3_args(p, k, r.req.origin[0], r.req.origin[1], r.req.origin[2], r.req.extent[0], r.req.extent[1],
                          r.req.extent[2], out, &d.a3s);
    } else if (p->dim == 2)
        general_args_2d(p, r.req.origin[0], r.req.origin[1], r.req.extent[0], r.req.extent[1], out, r.req.extent[0],
                        served_tile_h(s, p->smoothness), &d.a2);
    else
        general_args_3d(p, r.req.origin[0], r.req.origin[1], r.req.origin[2], r.req.extent[0], r.req.extent[1],
                        r.req.extent[2], out, &d.a3);
    if (r.lat) {
        d.lat_mode = phase == 1 ? 2 : 1;
        d.lat_n = r.lat_n;
        d.lat_host = s->lat_host + (size_t)slot * 2 * kMaxLatTbl;
        d.lat_base = s->arena_mem;
        for (int o = 0; o < kMaxOctaves; ++o) {
            d.lat_bx0[o] = r.lat_bx0[o];
            d.lat_by0[o] = r.lat_by0[o];
            d.lat_nbx[o] = r.lat_nbx[o];
            d.lat_tbl0[o] = r.lat_tbl0[o];
        }
    }
    std::memcpy(&s->reqs[slot], &d, sizeof(d));
    for (uint64_t i = 0; i < items; ++i) {
        ServeItem it;
        it.slot = (uint32_t)slot | (items == 1 ? kOnlyItem : 0u);
        it.seq = r.seq;
        const int64_t t0 = (int64_t)i * per;
        it.tile0 = (uint32_t)t0;
        it.ntiles = (uint32_t)std::min<int64_t>(per, nwork - t0);
        std::memcpy(&s->ring[(r.ring_begin + i) % (uint64_t)s->cfg.max_items], &it, sizeof(it));
    }
    s->tail = r.ring_end;
    std::atomic_thread_fence(std::memory_order_release);
    __atomic_store_n(&s->hc->tail, s->tail, __ATOMIC_RELEASE);
}

static bool ring_fits(const ptg_server *s, uint64_t items)
{
    return s->tail + items - s->reclaimed <= (uint64_t)s->cfg.max_items;
}

// Publish a waiting request's next phase if it can go: fills need ring space; tiles need
// ring space and every block they read written (by their own fills or another's).
static bool lat_try(ptg_server *s, uint64_t ticket, Request &r)
{
    if (r.lat_bad) {
        complete(s, ticket, PTG_EHIP);
        return true;
    }
    if (r.next_phase == 2 && r.lat_unready > 0) return false;
    if (!ring_fits(s, (uint64_t)(r.next_phase == 1 ? r.fill_items : r.items))) return false;
    publish(s, ticket, r, r.next_phase);
    return true;
}

static void lat_advance(ptg_server *s)
{
    for (size_t i = 0; i < s->lat_waiting.size();) {
        const uint64_t ticket = s->lat_waiting[i];
        if (lat_try(s, ticket, s->by_ticket[ticket]))
            s->lat_waiting.erase(s->lat_waiting.begin() + (ptrdiff_t)i);  // the others keep their order
        else
            ++i;
    }
}

static void admit(ptg_server *s)
{
    const int64_t now = now_ns();
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        Request &r = s->by_ticket[*it];
        // a strip is one wave's work: items of a strip request hold whole workgroups' worth
        const bool strips = r.kernel == PTG_TUNE_STRIP_2D || r.kernel == PTG_TUNE_STRIP_3D;
        r.per_item = strips ? kServeWaves * tiles_per_item(s, (r.ntiles + kServeWaves - 1) / kServeWaves)
                            : tiles_per_item(s, r.ntiles);
        r.items = (r.ntiles + r.per_item - 1) / r.per_item;
        const uint64_t items = (uint64_t)r.items;
        if (s->free_slots.empty()) break;
        if (!ring_fits(s, items)) break;  // ring order is FIFO
        const int64_t off = arena_alloc(s, round256(r.bytes));
        if (off < 0) {
            if (now - r.t_submit > kStarveNs) break;  // it waited long enough: nobody passes it
            ++it;
            continue;
        }
        r.arena_off = off;
        const uint64_t ticket = *it;
        r.slot = s->free_slots.back();
        s->free_slots.pop_back();
        if (r.lat && !lat_acquire(s, ticket, r)) {  // its missing blocks do not fit yet
            s->free_slots.push_back(r.slot);
            r.slot = -1;
            s->arena->release(r.arena_off, round256(r.bytes));
            r.arena_off = -1;
            if (now - r.t_submit > kStarveNs) break;
            ++it;
            continue;
        }
        it = s->pending.erase(it);
        s->tiles_pending -= work_units(r.kernel, r.ntiles);
        r.t_admit = now_ns();
        s->st.admitted++;
        if (r.lat) {
            r.next_phase = r.lat_fill.empty() ? 2 : 1;
            r.status = 4;
            if (!lat_try(s, ticket, r)) s->lat_waiting.push_back(ticket);
            continue;
        }
        publish(s, ticket, r, 2);
    }
}

static void poll_done(ptg_server *s)
{
    const int64_t now = now_ns();
    for (size_t i = 0; i < s->inflight.size();) {
        const uint64_t ticket = s->inflight[i];
        Request &r = s->by_ticket[ticket];
        const bool fin = s->gpu ? (__atomic_load_n(&s->done[r.slot], __ATOMIC_ACQUIRE) == r.seq) : (now >= r.fake_done_at);
        if (!fin) {
            ++i;
            continue;
        }
        s->inflight[i] = s->inflight.back();
        s->inflight.pop_back();
        if (r.status == 3) {  // fills done: the tiles follow
            lat_filled(s, r);
            span_done(s, ticket, 1);
            r.next_phase = 2;
            r.status = 4;
            s->lat_waiting.push_back(ticket);
            s->last_event = now;
        } else {
            complete(s, ticket, PTG_OK);
        }
    }
}

static void fail_inflight(ptg_server *s, int status)
{
    std::vector<uint64_t> all(s->inflight);
    all.insert(all.end(), s->lat_waiting.begin(), s->lat_waiting.end());
    s->inflight.clear();
    s->lat_waiting.clear();
    for (uint64_t t : all) complete(s, t, status);
}

// Kernel state: running (launched, not yet seen finished) and park_requested (ctl->park
// set, nothing is published until the kernel has left).
static void check_kernel(ptg_server *s)
{
    if (!s->gpu || !s->kernel_running) return;
    // the kernel only leaves after a park request (or on a fault): between those, query the
    // stream at most every kQueryNs so the scheduler loop stays fast (a query is a runtime call)
    const int64_t now = now_ns();
    if (!s->park_requested && now - s->last_query < kQueryNs) return;
    s->last_query = now;
    const hipError_t q = hipStreamQuery(s->stream);
    if (q == hipErrorNotReady) return;
    s->kernel_running = false;
    if (q != hipSuccess) {
        s->err = hipGetErrorString(q);
        fail_inflight(s, PTG_EHIP);
    } else if (!s->park_requested && !s->inflight.empty()) {
        s->err = "the serving kernel left with work in flight";
        fail_inflight(s, PTG_EHIP);
    }
    // every published item below tail has run (park is only set with nothing in flight,
    // or at shutdown after the in-flight set drained): the next launch starts at tail
    s->base = s->tail;
    s->park_requested = false;
    __atomic_store_n(&s->hc->park, 0, __ATOMIC_RELEASE);
}

static void ensure_kernel(ptg_server *s)
{
    if (!s->gpu || s->inflight.empty() || s->kernel_running || s->park_requested) return;
    hipLaunchKernelGGL(k_serve_reset, dim3(1), dim3(1), 0, s->stream, s->dc, s->base);
    hipLaunchKernelGGL(k_serve, dim3(s->workgroups), dim3(256), kServeLds, s->stream, s->hc, s->ring, s->reqs, s->done,
                       s->dc, s->cfg.max_items);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        s->err = hipGetErrorString(e);
        fail_inflight(s, PTG_EHIP);
        return;
    }
    s->kernel_running = true;
    s->st.kernel_launches++;
}

static void maybe_park(ptg_server *s, int64_t now)
{
    if (!s->gpu || !s->kernel_running || s->park_requested || !s->inflight.empty()) return;
    // requests still pending wait for arena bytes that only ptg_tile_release frees: they do
    // not keep the kernel (and with it a device-wide synchronisation) waiting
    if (!s->stopping && now - s->idle_since < kParkNs) return;
    s->park_requested = true;
    __atomic_store_n(&s->hc->park, 1, __ATOMIC_RELEASE);
}

static void service(ptg_server *s)
{
    if (s->gpu) (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        check_kernel(s);
        if (!s->park_requested) lat_advance(s);
        if (!s->stopping && !s->park_requested) admit(s);
        const bool busy = !s->inflight.empty();
        poll_done(s);
        if (!s->park_requested) lat_advance(s);
        const int64_t now = now_ns();
        if (busy && s->inflight.empty()) s->idle_since = now;
        ensure_kernel(s);
        maybe_park(s, now);
        if (s->stopping && s->inflight.empty() && s->lat_waiting.empty() && !s->kernel_running) break;
        // spin while requests are in flight or soon after the last event (completion is
        // seen within a poll, not a sleep); then sleep briefly while a kernel may still
        // need parking (releases that arrive meanwhile free their bytes together, and the
        // requests waiting for them are admitted together rather than one by one as each
        // release comes in), and block when there is nothing to do
        if (!s->inflight.empty() || !s->lat_waiting.empty() || now - s->last_event < kSpinNs) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else if (s->kernel_running) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            lk.lock();
        } else {
            s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

static int validate_req(const ptg_server *s, const ptg_tile_req *r, int64_t *bytes, int64_t *ntiles, int32_t *kernel,
                        int32_t *lat)
{
    const ptg_params *p = &r->params;
    if (!p || (p->dim != 2 && p->dim != 3)) return fail(PTG_EINVAL, "request dim must be 2 or 3");
    int rc = validate_params(p, p->dim);
    if (rc) return rc;
    if (p->form != PTG_FORM_PLAIN || p->out_dtype != PTG_F32)
        return fail(PTG_EINVAL, "served tiles use the plain form with FP32 output");
    if (p->model != PTG_MODEL_GRADIENT && p->model != PTG_MODEL_ZERO_GRADIENT && p->model != PTG_MODEL_HEIGHT_GRADIENT)
        return fail(PTG_EINVAL, "served tiles use the gradient, zero-gradient or height-and-gradient cells");
    if (p->smoothness > 3) return fail(PTG_EINVAL, "served tiles are C1, C2 or C3");
    const int nd = p->dim;
    for (int a = 0; a < 3; ++a) {
        if (a < nd) {
            if (r->extent[a] < 1) return fail(PTG_EINVAL, "request extent must be >= 1");
            if ((rc = validate_extent("tile", r->origin[a], r->extent[a]))) return rc;
        } else if (r->extent[a] != 1 || r->origin[a] != 0) {
            return fail(PTG_EINVAL, "a 2D request has extent[2] = 1 and origin[2] = 0");
        }
    }
    const int64_t nx = r->extent[0], ny = r->extent[1], nz = r->extent[2];
    if (nx > (1LL << 40) / ny || nx * ny > (1LL << 40) / nz) return fail(PTG_EINVAL, "request too large");
    *bytes = nx * ny * nz * 4;
    size_t lds;
    int k = 0;
    Fbm2dStripArgs sa;
    Fbm3dStripArgs sb;
    *kernel = nd == 2 ? PTG_TUNE_GENERAL_2D : PTG_TUNE_GENERAL_3D;
    const int hw = p->model == PTG_MODEL_HEIGHT_GRADIENT ? 1 : 0;  // node blocks also hold heights
    if (nd == 3 && p->smoothness <= 2 && dyadic_shift(p, &k) &&
        strip3_args(p, k, r->origin[0], r->origin[1], r->origin[2], nx, ny, nz, nullptr, &sb) == 0 &&
        (size_t)(kStrip3SharedWords + strip3_shared_words(sb.tab_total, sb.keys_col + 4 * sb.n_coarse, sb.nodes_listed) +
                 kServeWaves * strip3_wave_words(sb.nodes_total, sb.keys_total, hw)) * 4 <= kServeLds) {
        // dyadic ladder the 3D strip code takes (finest period >= 2) whose footprint fits a
        // serving workgroup
        *kernel = PTG_TUNE_STRIP_3D;
        *ntiles = sb.blocks;
        lds = 0;
    } else if (nd == 2 && dyadic_shift(p, &k) &&
        strip_args_2d(p, k, r->origin[0], r->origin[1], nx, ny, nullptr, nx, &sa) == 0 && sa.lo >= 1 &&
        (size_t)(kStripSharedWords + strip_shared_words(sa.nodes_hashed, sa.keys_total) +
                 kServeWaves * strip_wave_words(sa.nodes_total, sa.keys_total, hw)) * 4 <= kServeLds) {
        // dyadic ladder whose strip footprint fits a serving workgroup: the strip code
        *kernel = PTG_TUNE_STRIP_2D;
        *ntiles = sa.strips;
        lds = 0;
    } else if (nd == 2) {
        const int th = served_tile_h(s, p->smoothness);
        *ntiles = ((nx + kTile2 - 1) / kTile2) * ((ny + th - 1) / th);
        Fbm2dArgs ga;
        lds = general_args_2d(p, r->origin[0], r->origin[1], nx, ny, nullptr, nx, th, &ga);
    } else {
        *ntiles = ((nx + kTile3X - 1) / kTile3X) * ((ny + kTile3Y - 1) / kTile3Y) * ((nz + kTile3Z - 1) / kTile3Z);
        Fbm3dArgs ga;
        lds = general_args_3d(p, r->origin[0], r->origin[1], r->origin[2], nx, ny, nz, nullptr, &ga);
    }
    if (lds > kServeLds) return fail(PTG_EINVAL, "the request's lattice is too fine for a serving workgroup");
    if (*ntiles > 0x7FFFFFFFLL) return fail(PTG_EINVAL, "request too large");
    const int64_t per = (*kernel == PTG_TUNE_STRIP_2D || *kernel == PTG_TUNE_STRIP_3D ? kServeWaves : 1) *
                        (s->cfg.tiles_per_item > 0 ? s->cfg.tiles_per_item : kMaxTilesPerItem);
    const uint64_t items = (uint64_t)((*ntiles + per - 1) / per);
    if (items > (uint64_t)s->cfg.max_items) return fail(PTG_E2BIG, "request needs more work items than the ring holds");
    if (round256(*bytes) > s->cfg.hbm_budget_bytes)
        return fail(PTG_E2BIG, "request output (%lld bytes) exceeds the budget", (long long)*bytes);
    // lattice cache: general 2D requests whose blocks fit the table and, all missing, the
    // budget beside the output (others hash their nodes)
    *lat = 0;
    if (s->cfg.lattice_cache && *kernel == PTG_TUNE_GENERAL_2D && p->model == PTG_MODEL_GRADIENT) {
        const int n = lat_geometry(p, r->origin[0], r->origin[1], nx, ny, nullptr);
        if (n > 0 && round256(*bytes) + n * kLatBlockBytes <= s->cfg.hbm_budget_bytes) *lat = 1;
    }
    return PTG_OK;
}

static void free_server(ptg_server *s)
{
    if (s->gpu) {
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->lat_host) (void)hipHostFree(s->lat_host);
        if (s->hc) (void)hipHostFree(s->hc);
        if (s->ring) (void)hipHostFree(s->ring);
        if (s->reqs) (void)hipHostFree(s->reqs);
        if (s->done) (void)hipHostFree(s->done);
        if (s->dc) (void)hipFree(s->dc);
        if (s->arena_mem) (void)hipFree(s->arena_mem);
    } else {
        std::free(s->arena_mem);
    }
    delete s;
}

}  // namespace ptg

using namespace ptg;

extern "C" {

int ptg_server_create(const ptg_server_cfg *cfg, ptg_server **out)
{
    if (!cfg || !out) return fail(PTG_EINVAL, "NULL argument");
    if (cfg->hbm_budget_bytes <= 0) return fail(PTG_EINVAL, "hbm_budget_bytes must be > 0");
    if (cfg->max_items < 64 || cfg->max_items > (1 << 24)) return fail(PTG_EINVAL, "max_items must be in 64..2^24");
    if (cfg->workgroups < 0 || cfg->workgroups > 65536) return fail(PTG_EINVAL, "bad workgroup count");
    if (cfg->executor != PTG_EXEC_GPU && cfg->executor != PTG_EXEC_HOST) return fail(PTG_EINVAL, "bad executor");
    if (cfg->executor == PTG_EXEC_HOST && cfg->fake_tile_ns < 0) return fail(PTG_EINVAL, "fake_tile_ns < 0");
    if (cfg->tiles_per_item < 0 || cfg->tiles_per_item > kMaxTilesPerItem)
        return fail(PTG_EINVAL, "tiles_per_item must be in 0..%d", kMaxTilesPerItem);
    if ((cfg->autotune != 0 && cfg->autotune != 1) || (cfg->lattice_cache != 0 && cfg->lattice_cache != 1))
        return fail(PTG_EINVAL, "autotune and lattice_cache must be 0 or 1");
    if (cfg->tile_h != 0 && cfg->tile_h != 16 && cfg->tile_h != 32 && cfg->tile_h != 64)
        return fail(PTG_EINVAL, "tile_h must be 0, 16, 32 or 64");
    if (cfg->lattice_cache && cfg->hbm_budget_bytes > (int64_t(1) << 40))
        return fail(PTG_EINVAL, "lattice_cache needs a budget of at most 1 TiB");
    if (cfg->autotune && cfg->executor == PTG_EXEC_GPU && cfg->hbm_budget_bytes < (1 << 20))
        return fail(PTG_EINVAL, "autotune needs a budget of at least 1 MiB");
    *out = nullptr;
    ptg_server *s = new ptg_server();
    s->cfg = *cfg;
    s->gpu = cfg->executor == PTG_EXEC_GPU;
    s->st.budget = cfg->hbm_budget_bytes;
    for (int i = kReqSlots - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->slot_total.assign(kReqSlots, 0);
    s->arena.reset(new Arena(cfg->hbm_budget_bytes));
    if (cfg->tile_h != 0) s->tile_h2[0] = s->tile_h2[1] = cfg->tile_h;
    s->workgroups = cfg->workgroups > 0 ? cfg->workgroups : 256;
    if (s->gpu) {
        hipError_t e = hipSetDevice(cfg->device);
        if (e != hipSuccess) {
            free_server(s);
            return hip_fail(e, "hipSetDevice");
        }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device) != hipSuccess || cus <= 0)
            cus = 256;
        // one per compute unit: a request with fewer items than workgroups then spreads one item
        // per unit (two on one unit would share it while others idle); capacity is the same
        s->workgroups = cfg->workgroups > 0 ? cfg->workgroups : cus;
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e == hipSuccess && cfg->lattice_cache)
            e = hipHostMalloc((void **)&s->lat_host, sizeof(uint32_t) * 2 * kMaxLatTbl * kReqSlots,
                              hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s->hc, sizeof(ServeHostCtl), hipHostMallocCoherent);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&s->ring, sizeof(ServeItem) * (size_t)cfg->max_items, hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s->reqs, sizeof(ServeReqDesc) * kReqSlots, hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s->done, sizeof(uint32_t) * kReqSlots, hipHostMallocCoherent);
        if (e == hipSuccess) e = hipMalloc((void **)&s->dc, sizeof(ServeDevCtl));
        if (e == hipSuccess) e = hipMemset(s->dc, 0, sizeof(ServeDevCtl));
        if (e == hipSuccess) e = hipMalloc((void **)&s->arena_mem, (size_t)cfg->hbm_budget_bytes);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_serve),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kServeLds);
        if (e != hipSuccess) {
            const int code = (e == hipErrorOutOfMemory) ? PTG_ENOMEM : PTG_EHIP;
            hip_fail(e, "server allocation");
            free_server(s);
            return code;
        }
        std::memset(s->hc, 0, sizeof(ServeHostCtl));
        std::memset(s->done, 0, sizeof(uint32_t) * kReqSlots);
        if (cfg->autotune && cfg->tile_h == 0) {  // tile heights timed on the arena, before any request
            for (int m = 1; m <= 2; ++m) {
                ptg_params p;
                ptg_params_default(&p);
                p.smoothness = m;
                p.base_freq = 1.0 / 4096.0;
                p.path = PTG_PATH_GENERAL;
                ptg_tune_result r;
                const int rc = ptg_tune_2d(&p, 0, 0, 512, 512, s->arena_mem, 512, s->stream, 5, &r);
                if (rc != PTG_OK) {
                    free_server(s);
                    return rc;
                }
                // the serving kernel takes tiles of at most kTile2 rows: the fastest of those
                int best = -1;
                for (int i = 0; i < r.n; ++i)
                    if (r.candidates[i] <= kTile2 && (best < 0 || r.us[i] < r.us[best])) best = i;
                s->tile_h2[m - 1] = best >= 0 ? r.candidates[best] : kTile2;
            }
        }
    } else {
        s->arena_mem = static_cast<char *>(std::malloc((size_t)cfg->hbm_budget_bytes));
        if (!s->arena_mem) {
            free_server(s);
            return fail(PTG_ENOMEM, "arena allocation");
        }
    }
    s->th = std::thread(service, s);
    *out = s;
    return PTG_OK;
}

int ptg_tiles_submit(ptg_server *s, const ptg_tile_req *reqs, int32_t n, uint64_t *tickets_out)
{
    if (!s || (n > 0 && (!reqs || !tickets_out)) || n < 0) return fail(PTG_EINVAL, "bad arguments");
    std::vector<int64_t> bytes(n), tiles(n);
    std::vector<int32_t> kernels(n);
    std::vector<int32_t> lat(n);
    for (int32_t i = 0; i < n; ++i) {
        const int rc = validate_req(s, &reqs[i], &bytes[i], &tiles[i], &kernels[i], &lat[i]);
        if (rc) return rc;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(PTG_ESHUTDOWN, "server is shutting down");
    const int64_t t = now_ns();
    s->last_event = t;
    for (int32_t i = 0; i < n; ++i) {
        const uint64_t ticket = s->next_ticket++;
        Request &r = s->by_ticket[ticket];
        r.req = reqs[i];
        r.bytes = bytes[i];
        r.ntiles = tiles[i];
        r.kernel = kernels[i];
        r.lat = lat[i];
        r.t_submit = t;
        s->pending.push_back(ticket);
        s->tiles_pending += work_units(r.kernel, r.ntiles);
        tickets_out[i] = ticket;
        s->st.submitted++;
    }
    // admit at once on this thread when the scheduler would (saves its wake-up); it still
    // launches the kernel, polls completions and retries what does not fit
    if (!s->park_requested) admit(s);
    s->cv_work.notify_all();
    return PTG_OK;
}

static void fill_result(const ptg_server *s, const Request &r, ptg_tile_result *res)
{
    std::memset(res, 0, sizeof(*res));
    res->status = r.status;
    res->kernel = r.kernel;
    res->out_dev = (r.status == PTG_OK) ? s->arena_mem + r.arena_off : nullptr;
    res->bytes = r.bytes;
    res->user_tag = r.req.user_tag;
    res->t_submit_ns = r.t_submit;
    res->t_admit_ns = r.t_admit;
    res->t_done_ns = r.t_done;
}

// The pending request at the head of admission waits for arena bytes that only the caller
// can free: nothing is in flight (nothing will complete and free bytes), completed outputs
// still hold arena bytes, and the largest free range is too small for it.
static bool head_blocked_by_caller(const ptg_server *s, uint64_t ticket)
{
    auto j = s->by_ticket.find(ticket);
    if (j == s->by_ticket.end() || j->second.status != 1 || !s->inflight.empty()) return false;
    bool held = false;
    for (const auto &kv : s->by_ticket)
        if (kv.second.status <= 0 && kv.second.arena_off >= 0) {
            held = true;
            break;
        }
    return held && s->arena->largest_free() < round256(j->second.bytes);
}

int ptg_tiles_wait(ptg_server *s, uint64_t ticket, int64_t timeout_ns, ptg_tile_result *res)
{
    if (!s || !res) return fail(PTG_EINVAL, "bad arguments");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) return fail(PTG_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    auto ready = [&] {
        auto j = s->by_ticket.find(ticket);
        return j == s->by_ticket.end() || j->second.status <= 0;
    };
    auto blocked_by_caller = [&] { return head_blocked_by_caller(s, ticket); };
    // wait in slices; the blocked state must last across a slice (the scheduler makes an
    // admission pass in well under one) before it is reported
    const auto slice = std::chrono::milliseconds(2);
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns < 0 ? 0 : timeout_ns);
    bool was_blocked = false;
    while (!ready()) {
        if (timeout_ns == 0) break;
        auto until = std::chrono::steady_clock::now() + slice;
        if (timeout_ns > 0 && until > t_end) until = t_end;
        s->cv_done.wait_until(lk, until, ready);
        if (ready()) break;
        const bool b = blocked_by_caller();
        if (b && was_blocked)
            return fail(PTG_EAGAIN, "ticket %llu waits for arena bytes held by completed outputs that have not been "
                                    "released (release some, then wait again)",
                        (unsigned long long)ticket);
        was_blocked = b;
        if (timeout_ns > 0 && std::chrono::steady_clock::now() >= t_end) break;
    }
    it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) return fail(PTG_ENOENT, "ticket released");
    const Request &r = it->second;
    if (r.status > 0) return fail(PTG_ETIMEDOUT, "request still pending");
    fill_result(s, r, res);
    return PTG_OK;
}

int ptg_tiles_wait_any(ptg_server *s, int64_t timeout_ns, uint64_t *ticket_out, ptg_tile_result *res)
{
    if (!s || !res || !ticket_out) return fail(PTG_EINVAL, "bad arguments");
    std::unique_lock<std::mutex> lk(s->mu);
    // completions already released through their ticket are dropped from the queue
    auto ready = [&] {
        while (!s->done_q.empty() && s->by_ticket.find(s->done_q.front()) == s->by_ticket.end())
            s->done_q.pop_front();
        return !s->done_q.empty();
    };
    // nothing left that could complete: no request pending or in flight
    auto idle = [&] { return s->pending.empty() && s->inflight.empty() && s->lat_waiting.empty(); };
    const auto slice = std::chrono::milliseconds(2);
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns < 0 ? 0 : timeout_ns);
    bool was_blocked = false;
    while (!ready()) {
        if (idle()) return fail(PTG_ENOENT, "no request is pending or in flight");
        if (timeout_ns == 0) return fail(PTG_ETIMEDOUT, "no request completed");
        auto until = std::chrono::steady_clock::now() + slice;
        if (timeout_ns > 0 && until > t_end) until = t_end;
        s->cv_done.wait_until(lk, until, ready);
        if (ready()) break;
        const bool b = !s->pending.empty() && head_blocked_by_caller(s, s->pending.front());
        if (b && was_blocked)
            return fail(PTG_EAGAIN, "the pending requests wait for arena bytes held by completed outputs that have "
                                    "not been released (release some, then wait again)");
        was_blocked = b;
        if (timeout_ns > 0 && std::chrono::steady_clock::now() >= t_end)
            return fail(PTG_ETIMEDOUT, "no request completed");
    }
    const uint64_t t = s->done_q.front();
    s->done_q.pop_front();
    *ticket_out = t;
    fill_result(s, s->by_ticket.find(t)->second, res);
    return PTG_OK;
}

int ptg_tile_release(ptg_server *s, uint64_t ticket)
{
    if (!s) return fail(PTG_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) return fail(PTG_ENOENT, "unknown ticket");
    if (it->second.status > 0) return fail(PTG_EAGAIN, "request not complete");
    if (it->second.arena_off >= 0) s->arena->release(it->second.arena_off, round256(it->second.bytes));
    s->by_ticket.erase(it);
    while (!s->done_q.empty() && s->by_ticket.find(s->done_q.front()) == s->by_ticket.end()) s->done_q.pop_front();
    s->st.released++;
    s->st.bytes_in_use = s->arena->used();
    s->cv_work.notify_all();
    return PTG_OK;
}

int ptg_server_stats_get(ptg_server *s, ptg_server_stats *st)
{
    if (!s || !st) return fail(PTG_EINVAL, "bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->st;
    st->pending = (int64_t)s->pending.size();
    st->in_flight = (int64_t)s->inflight.size();
    st->bytes_in_use = s->arena->used();
    st->lat_blocks = (int64_t)s->lat_cache.size();
    st->lat_bytes = st->lat_blocks * kLatBlockBytes;
    st->tile_h[0] = s->tile_h2[0];
    st->tile_h[1] = s->tile_h2[1];
    return PTG_OK;
}

int ptg_server_destroy(ptg_server *s)
{
    if (!s) return fail(PTG_EINVAL, "NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        for (uint64_t t : s->pending) complete(s, t, PTG_ESHUTDOWN);
        s->pending.clear();
        s->tiles_pending = 0;
        s->cv_work.notify_all();
    }
    s->th.join();  // in-flight requests run out, then the kernel is parked and has left
    int rc = PTG_OK;
    if (s->gpu) {
        const hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) rc = hip_fail(e, "server kernel");
    }
    free_server(s);
    return rc;
}

}  // extern "C"
