// ptg_graph.hip -- batches of dense-field calls launched as HIP graphs (a6): the graph of a
// batch shape is instantiated once and its kernel nodes' arguments are updated in place for
// every later batch of the same shape.
#include <list>
#include <map>
#include <vector>

#include "../../include/ptg.h"
#include "ptg_internal.h"
#include "ptg_launch.h"

namespace ptg {

LaunchSink *&launch_sink()
{
    static thread_local LaunchSink *sink = nullptr;
    return sink;
}

namespace {

constexpr int kInstPerShape = 4;   // instances of one shape (so none is updated while in flight)
constexpr size_t kMaxShapes = 64;  // shapes cached per batch object

// One instantiated graph of a shape: its kernel nodes in record order, and the event
// recorded after its last launch.
struct Inst {
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    std::vector<hipGraphNode_t> nodes;
    hipEvent_t ev = nullptr;
    bool launched = false;
};

struct Shape {
    std::list<Inst> insts;
    uint64_t last_use = 0;
    size_t next = 0;  // round robin when every instance is in flight
};

using Key = std::vector<uint64_t>;

// A batch's shape is its sequence of kernels (function, workgroup size, argument bytes); the
// grid, the dynamic LDS size and the arguments of a node are updated in place, so batches of
// the same kernels over fields of other sizes or origins reuse the instance.
Key shape_key(const std::vector<LaunchRec> &recs)
{
    Key k;
    k.reserve(recs.size() * 3);
    for (const LaunchRec &r : recs) {
        k.push_back(reinterpret_cast<uint64_t>(r.func));
        k.push_back(((uint64_t)r.block.x << 32) | ((uint64_t)r.block.y << 16) | r.block.z);
        k.push_back(r.arg_bytes);
    }
    return k;
}

hipKernelNodeParams node_params(const LaunchRec &r, void **argv)
{
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(r.func);
    kp.gridDim = r.grid;
    kp.blockDim = r.block;
    kp.sharedMemBytes = r.lds;
    argv[0] = const_cast<unsigned char *>(r.args);
    kp.kernelParams = argv;
    kp.extra = nullptr;
    return kp;
}

void free_inst(Inst &in)
{
    if (in.launched && in.ev) (void)hipEventSynchronize(in.ev);
    if (in.ex) (void)hipGraphExecDestroy(in.ex);
    if (in.g) (void)hipGraphDestroy(in.g);
    if (in.ev) (void)hipEventDestroy(in.ev);
    in = Inst{};
}

}  // namespace
}  // namespace ptg

struct ptg_batch {
    int32_t max_calls = 0;
    std::vector<ptg::LaunchRec> recs;
    std::map<ptg::Key, ptg::Shape> shapes;
    uint64_t clock = 0;
    ptg_batch_stats st{};
};

using namespace ptg;

namespace {

// Record the one launch of a dense-field call into the batch (validation as the direct call).
template <typename F>
int record(ptg_batch *b, F call)
{
    if (!b) return fail(PTG_EINVAL, "batch is NULL");
    if ((int32_t)b->recs.size() >= b->max_calls)
        return fail(PTG_EINVAL, "batch is full (%d calls)", (int)b->max_calls);
    LaunchSink sink{};
    sink.n = 0;
    LaunchSink *prev = launch_sink();
    launch_sink() = &sink;
    const int rc = call();
    launch_sink() = prev;
    if (rc != PTG_OK) return rc;
    if (sink.n > 1) return fail(PTG_EHIP, "a dense-field call made %d launches", sink.n);
    if (sink.n == 1) b->recs.push_back(sink.rec);
    return PTG_OK;
}

int new_inst(const std::vector<LaunchRec> &recs, Inst &in)
{
    hipError_t e = hipGraphCreate(&in.g, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphCreate");
    in.nodes.resize(recs.size());
    for (size_t i = 0; i < recs.size(); ++i) {
        void *argv[1];
        const hipKernelNodeParams kp = node_params(recs[i], argv);
        e = hipGraphAddKernelNode(&in.nodes[i], in.g, nullptr, 0, &kp);
        if (e != hipSuccess) return hip_fail(e, "hipGraphAddKernelNode");
    }
    e = hipGraphInstantiate(&in.ex, in.g, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    e = hipEventCreateWithFlags(&in.ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    return PTG_OK;
}

void evict_lru(ptg_batch *b)
{
    auto victim = b->shapes.begin();
    for (auto it = b->shapes.begin(); it != b->shapes.end(); ++it)
        if (it->second.last_use < victim->second.last_use) victim = it;
    for (Inst &in : victim->second.insts) free_inst(in);
    b->shapes.erase(victim);
}

}  // namespace

extern "C" {

int ptg_batch_create(int32_t max_calls, ptg_batch **out)
{
    if (!out) return fail(PTG_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_calls < 1 || max_calls > 4096) return fail(PTG_EINVAL, "max_calls must be in 1..4096");
    ptg_batch *b = new (std::nothrow) ptg_batch();
    if (!b) return fail(PTG_ENOMEM, "batch allocation");
    b->max_calls = max_calls;
    b->recs.reserve((size_t)max_calls);
    *out = b;
    return PTG_OK;
}

int ptg_batch_add_2d(ptg_batch *b, const ptg_params *p, int64_t x0, int64_t y0, int64_t nx, int64_t ny,
                     void *out_dev, int64_t row_pitch)
{
    return record(b, [&] { return ptg_fbm_2d(p, x0, y0, nx, ny, out_dev, row_pitch, nullptr); });
}

int ptg_batch_add_3d(ptg_batch *b, const ptg_params *p, int64_t x0, int64_t y0, int64_t z0, int64_t nx, int64_t ny,
                     int64_t nz, void *out_dev)
{
    return record(b, [&] { return ptg_fbm_3d(p, x0, y0, z0, nx, ny, nz, out_dev, nullptr); });
}

int ptg_batch_clear(ptg_batch *b)
{
    if (!b) return fail(PTG_EINVAL, "batch is NULL");
    b->recs.clear();
    return PTG_OK;
}

int ptg_batch_launch(ptg_batch *b, void *stream)
{
    if (!b) return fail(PTG_EINVAL, "batch is NULL");
    if (b->recs.empty()) return PTG_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Key key = shape_key(b->recs);
    auto it = b->shapes.find(key);
    if (it == b->shapes.end()) {
        if (b->shapes.size() >= kMaxShapes) evict_lru(b);
        it = b->shapes.emplace(key, Shape{}).first;
    }
    Shape &sh = it->second;
    sh.last_use = ++b->clock;
    // an instance that is idle (never launched, or its last launch has finished)
    Inst *use = nullptr;
    for (Inst &in : sh.insts)
        if (!in.launched || hipEventQuery(in.ev) == hipSuccess) {
            use = &in;
            break;
        }
    bool fresh = false;
    if (!use && (int)sh.insts.size() < kInstPerShape) {
        sh.insts.emplace_back();
        use = &sh.insts.back();
        const int rc = new_inst(b->recs, *use);
        if (rc != PTG_OK) {
            free_inst(*use);
            sh.insts.pop_back();
            b->recs.clear();
            return rc;
        }
        fresh = true;
        b->st.instantiations++;
    }
    if (!use) {  // every instance in flight: wait for the next one in turn
        auto in = sh.insts.begin();
        std::advance(in, (long)(sh.next++ % sh.insts.size()));
        use = &*in;
        const hipError_t e = hipEventSynchronize(use->ev);
        if (e != hipSuccess) {
            b->recs.clear();
            return hip_fail(e, "hipEventSynchronize");
        }
    }
    if (!fresh) {
        hipError_t e = hipSuccess;
        for (size_t i = 0; i < b->recs.size() && e == hipSuccess; ++i) {
            void *argv[1];
            const hipKernelNodeParams kp = node_params(b->recs[i], argv);
            e = hipGraphExecKernelNodeSetParams(use->ex, use->nodes[i], &kp);
        }
        if (e == hipSuccess) {
            b->st.updates++;
        } else {  // the runtime refused the update: instantiate this instance again
            (void)hipGetLastError();
            free_inst(*use);  // idle: its last launch has finished
            const int rc = new_inst(b->recs, *use);
            if (rc != PTG_OK) {
                b->recs.clear();
                return rc;
            }
            b->st.instantiations++;
        }
    }
    hipError_t e = hipGraphLaunch(use->ex, s);
    if (e == hipSuccess) e = hipEventRecord(use->ev, s);
    const int64_t n = (int64_t)b->recs.size();
    b->recs.clear();
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    use->launched = true;
    b->st.launches++;
    b->st.nodes += n;
    return PTG_OK;
}

int ptg_batch_stats_get(const ptg_batch *b, ptg_batch_stats *st)
{
    if (!b || !st) return fail(PTG_EINVAL, "NULL argument");
    *st = b->st;
    st->pending = (int64_t)b->recs.size();
    int64_t n = 0;
    for (const auto &kv : b->shapes) n += (int64_t)kv.second.insts.size();
    st->instances = n;
    return PTG_OK;
}

int ptg_batch_destroy(ptg_batch *b)
{
    if (!b) return fail(PTG_EINVAL, "batch is NULL");
    for (auto &kv : b->shapes)
        for (Inst &in : kv.second.insts) free_inst(in);
    delete b;
    return PTG_OK;
}

}  // extern "C"
