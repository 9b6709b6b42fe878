// ptg_loadgen.cpp -- open-loop load generation for terrain-tile streams: the same request
// stream with given arrival times driven through (a) the tile server and (b) the plain
// per-tile path (one ptg_fbm_2d / ptg_fbm_3d call per request on one stream, launched
// directly or in batches as HIP graphs through the library's ptg_batch).  Native threads issue and complete
// requests at their arrival times, so the measured latencies are those of the paths, not
// of an interpreter.  Benchmark support; not part of the library's C ABI.
#include "ptg_loadgen.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Sleep through most of the wait, spin the last 100 us.
void wait_until(int64_t t)
{
    for (;;) {
        const int64_t d = t - now_ns();
        if (d <= 0) return;
        if (d > 150000)
            std::this_thread::sleep_for(std::chrono::nanoseconds(d - 100000));
        else
            std::this_thread::yield();
    }
}

bool arrivals_ok(const int64_t *a, int32_t n)
{
    for (int32_t i = 0; i < n; ++i)
        if (a[i] < 0 || (i > 0 && a[i] < a[i - 1])) return false;
    return true;
}

int plain_call(const ptg_tile_req &r, void *out, hipStream_t s)
{
    if (r.params.dim == 2)
        return ptg_fbm_2d(&r.params, r.origin[0], r.origin[1], r.extent[0], r.extent[1], out, r.extent[0], s);
    return ptg_fbm_3d(&r.params, r.origin[0], r.origin[1], r.origin[2], r.extent[0], r.extent[1], r.extent[2], out, s);
}

}  // namespace

extern "C" {

int ptg_lg_served(ptg_server *s, const ptg_tile_req *reqs, const int64_t *arrival_ns, int32_t n, int64_t *done_ns,
                  int64_t *admit_ns, int32_t any_order)
{
    if (!s || !reqs || !arrival_ns || !done_ns || n < 1 || !arrivals_ok(arrival_ns, n)) return PTG_EINVAL;
    std::vector<uint64_t> tickets((size_t)n);
    std::atomic<int32_t> published{0};
    std::atomic<int> err{PTG_OK};
    const int64_t t0 = now_ns() + 1000000;
    std::thread sub([&] {
        int32_t i = 0;
        while (i < n && err.load() == PTG_OK) {
            wait_until(t0 + arrival_ns[i]);
            const int64_t now = now_ns();
            int32_t j = i + 1;
            while (j < n && t0 + arrival_ns[j] <= now) ++j;
            const int rc = ptg_tiles_submit(s, reqs + i, j - i, tickets.data() + i);
            if (rc != PTG_OK) {
                err.store(rc);
                break;
            }
            published.store(j, std::memory_order_release);
            i = j;
        }
    });
    int rc = PTG_OK;
    if (!any_order) {
        std::vector<char> taken((size_t)n, 0);
        auto take = [&](int32_t k, const ptg_tile_result &res) {
            int r = res.status;
            if (r == PTG_OK) {
                done_ns[k] = res.t_done_ns - t0;
                if (admit_ns) admit_ns[k] = res.t_admit_ns - t0;
                r = ptg_tile_release(s, tickets[(size_t)k]);
            }
            taken[(size_t)k] = 1;
            return r;
        };
        for (int32_t i = 0; i < n && rc == PTG_OK; ++i) {
            if (taken[(size_t)i]) continue;
            while (published.load(std::memory_order_acquire) <= i) {
                if (err.load() != PTG_OK) break;
                std::this_thread::yield();
            }
            if (err.load() != PTG_OK) {
                rc = err.load();
                break;
            }
            ptg_tile_result res;
            rc = ptg_tiles_wait(s, tickets[(size_t)i], 120000000000LL, &res);
            while (rc == PTG_EAGAIN) {
                // request i waits for bytes held by later requests that completed first: take
                // (and release) those, then wait again
                const int32_t pub = published.load(std::memory_order_acquire);
                for (int32_t k = i + 1; k < pub && rc == PTG_EAGAIN; ++k) {
                    if (taken[(size_t)k]) continue;
                    ptg_tile_result rk;
                    if (ptg_tiles_wait(s, tickets[(size_t)k], 0, &rk) == PTG_OK) {
                        const int rt = take(k, rk);
                        if (rt != PTG_OK) rc = rt;
                    }
                }
                if (rc == PTG_EAGAIN) rc = ptg_tiles_wait(s, tickets[(size_t)i], 120000000000LL, &res);
            }
            if (rc == PTG_OK) rc = take(i, res);
        }
    } else {
        // completions in completion order; a ticket is mapped back to its request by its place
        // in tickets[] (increasing in submission order)
        for (int32_t taken = 0; taken < n && rc == PTG_OK; ++taken) {
            uint64_t t = 0;
            ptg_tile_result res;
            for (;;) {
                rc = ptg_tiles_wait_any(s, 2000000LL, &t, &res);
                if (rc != PTG_ENOENT && rc != PTG_ETIMEDOUT) break;
                // still running, or nothing submitted yet (the next arrival is ahead): wait on,
                // unless submission failed
                if (err.load() != PTG_OK) {
                    rc = err.load();
                    break;
                }
                if (rc == PTG_ENOENT) std::this_thread::sleep_for(std::chrono::microseconds(20));
                rc = PTG_OK;
            }
            if (rc != PTG_OK) break;
            int32_t i = -1;
            while (i < 0) {  // the submitting thread publishes tickets[] after the submit call returns
                const int32_t pub = published.load(std::memory_order_acquire);
                const auto it = std::lower_bound(tickets.begin(), tickets.begin() + pub, t);
                if (it != tickets.begin() + pub && *it == t) i = (int32_t)(it - tickets.begin());
                else std::this_thread::yield();
            }
            if (res.status != PTG_OK) {
                rc = res.status;
                break;
            }
            done_ns[i] = res.t_done_ns - t0;
            if (admit_ns) admit_ns[i] = res.t_admit_ns - t0;
            rc = ptg_tile_release(s, t);
        }
    }
    if (rc != PTG_OK) err.store(rc);
    sub.join();
    return rc;
}

int ptg_lg_plain(const ptg_tile_req *reqs, const int64_t *arrival_ns, int32_t n, void *arena, int64_t arena_bytes,
                 int32_t mode, int32_t max_batch, int64_t *done_ns, int64_t *stats)
{
    // Graph mode is switched off: one stream of thousands of one-request graph launches with
    // in-place node updates ended the process with a segmentation fault whose cause has not
    // been established (the batch object's own use of the graph API has been checked by
    // reading; its GPU tests pass).  The code below stays for when the cause is known.
    if (mode == PTG_LG_GRAPH) return PTG_EINVAL;
    if (!reqs || !arrival_ns || !done_ns || !arena || n < 1 || !arrivals_ok(arrival_ns, n) ||
        (mode != PTG_LG_DIRECT && mode != PTG_LG_SOLO) || max_batch < 1)
        return PTG_EINVAL;
    std::vector<int64_t> off((size_t)n);
    int64_t o = 0;
    for (int32_t i = 0; i < n; ++i) {  // outputs laid out in arrival order, wrapping (one stream orders reuse)
        int64_t b = reqs[i].extent[0] * reqs[i].extent[1] * reqs[i].extent[2] * 4;
        b = (b + 255) & ~int64_t(255);
        if (b > arena_bytes) return PTG_E2BIG;
        if (o + b > arena_bytes) o = 0;
        off[(size_t)i] = o;
        o += b;
    }
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return PTG_EHIP;
    if (mode == PTG_LG_SOLO) {  // each request alone: its kernel time between two events
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int rc = (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) ? PTG_OK : PTG_EHIP;
        for (int32_t i = 0; i < n && rc == PTG_OK; ++i) {
            if (hipEventRecord(e0, st) != hipSuccess) rc = PTG_EHIP;
            if (rc == PTG_OK) rc = plain_call(reqs[i], (char *)arena + off[(size_t)i], st);
            if (rc == PTG_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rc = PTG_EHIP;
            float ms = 0.0f;
            if (rc == PTG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = PTG_EHIP;
            done_ns[i] = (int64_t)((double)ms * 1e6);
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(st);
        if (stats) {
            stats[0] = n;
            stats[1] = stats[2] = 0;
        }
        return rc;
    }
    // graph mode: the library's batch object (instantiates a graph once per batch shape and
    // updates its arguments for later batches of that shape)
    ptg_batch *batch = nullptr;
    if (mode == PTG_LG_GRAPH && ptg_batch_create(max_batch, &batch) != PTG_OK) {
        (void)hipStreamDestroy(st);
        return PTG_EHIP;
    }
    // one completion event per launch unit (a request, or a batch)
    std::vector<hipEvent_t> ev((size_t)n, nullptr);
    for (auto &e : ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            for (auto &f : ev)
                if (f) (void)hipEventDestroy(f);
            if (batch) (void)ptg_batch_destroy(batch);
            (void)hipStreamDestroy(st);
            return PTG_EHIP;
        }
    std::vector<int32_t> unit_end((size_t)n, 0);     // unit u covers requests [u, unit_end[u])
    std::atomic<int32_t> issued{0};                  // requests whose unit has been launched
    std::atomic<int> err{PTG_OK};
    int64_t launches = 0;
    const int64_t t0 = now_ns() + 1000000;
    std::thread wt([&] {  // completion side: units finish in stream order
        int32_t u = 0;
        while (u < n) {
            while (issued.load(std::memory_order_acquire) <= u) {
                if (err.load() != PTG_OK) return;
                std::this_thread::yield();
            }
            if (hipEventSynchronize(ev[(size_t)u]) != hipSuccess) {
                err.store(PTG_EHIP);
                return;
            }
            const int64_t t = now_ns() - t0;
            const int32_t e = unit_end[(size_t)u];
            for (int32_t k = u; k < e; ++k) done_ns[k] = t;
            u = e;
        }
    });
    int32_t i = 0;
    while (i < n && err.load() == PTG_OK) {
        wait_until(t0 + arrival_ns[i]);
        int rc = PTG_OK;
        int32_t j = i + 1;
        if (mode == PTG_LG_DIRECT) {
            rc = plain_call(reqs[i], (char *)arena + off[(size_t)i], st);
        } else {  // every request that has arrived, up to max_batch, in one graph launch
            const int64_t now = now_ns();
            while (j < n && j - i < max_batch && t0 + arrival_ns[j] <= now) ++j;
            for (int32_t k = i; k < j && rc == PTG_OK; ++k) {
                const ptg_tile_req &r = reqs[k];
                void *out = (char *)arena + off[(size_t)k];
                rc = r.params.dim == 2
                         ? ptg_batch_add_2d(batch, &r.params, r.origin[0], r.origin[1], r.extent[0], r.extent[1], out,
                                            r.extent[0])
                         : ptg_batch_add_3d(batch, &r.params, r.origin[0], r.origin[1], r.origin[2], r.extent[0],
                                            r.extent[1], r.extent[2], out);
            }
            if (rc == PTG_OK) rc = ptg_batch_launch(batch, st);
        }
        if (rc == PTG_OK && hipEventRecord(ev[(size_t)i], st) != hipSuccess) rc = PTG_EHIP;
        if (rc != PTG_OK) {
            err.store(rc);
            break;
        }
        ++launches;
        unit_end[(size_t)i] = j;
        issued.store(j, std::memory_order_release);
        i = j;
    }
    wt.join();
    if (hipStreamSynchronize(st) != hipSuccess && err.load() == PTG_OK) err.store(PTG_EHIP);
    ptg_batch_stats bs{};
    if (batch) {
        (void)ptg_batch_stats_get(batch, &bs);
        (void)ptg_batch_destroy(batch);
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(st);
    if (stats) {
        stats[0] = launches;
        stats[1] = bs.instantiations;
        stats[2] = bs.updates;
    }
    return err.load();
}

}  // extern "C"
