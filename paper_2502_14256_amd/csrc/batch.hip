// Batched fit of an instance table (Sec. 6 solves many randomizations and
// right-hand sides together, vectorised over them): an instance is one
// randomized point set (a scramble and shift of its own, one shared
// generating vector or matrix per kind) with n = 2^m points and nrhs
// responses.  The plan groups the table by (kind, m, nrhs); the instances of
// a group are the replications of one point set, so each group costs one
// first-column launch and one fit (eigenvalues, every solve and the
// log-det).  Groups are shared out over the plan's streams (fork/join through
// events on the caller's stream), and the whole sequence can be captured as
// one HIP graph that every later launch replays.
//
// The data live in caller-owned arenas laid out by the plan (every group's
// rows contiguous); the per-group point-set data (shifts, scrambles, each
// net replication's scrambled columns), the first columns and the fit
// workspaces live in the caller's workspace arena.  The plan itself holds
// host memory, its streams, events and graph only.
#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace ldk {
namespace {

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Group {
    int kind, m, nrhs, R;
    std::vector<int> members;  // table indices, in row order
    size_t y_off, lam_off, ld_off;          // elements (y/c: dtype; lam/logdet: double)
    size_t ws_shift, ws_lms, ws_cols, ws_k1, ws_fit;  // byte offsets in the workspace arena
    size_t fit_bytes;
};

}  // namespace
}  // namespace ldk

struct ldk_plan_s {
    ldk_batch_desc desc;
    std::vector<int32_t> alpha_lat, alpha_net;
    std::vector<ldk_instance> inst;
    std::vector<ldk::Group> groups;
    std::vector<std::pair<int, int>> where;  // instance -> (group, row)
    size_t arena[LDK_ARENA_COUNT];
    // bound arenas
    void *y = nullptr, *c = nullptr, *ws = nullptr;
    double *lam = nullptr, *logdet = nullptr;
    bool bound = false;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;  // [0]: fork; [1 + s]: join of stream s
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace ldk {
namespace {

size_t esz(int dtype) { return dtype == LDK_F64 ? 8 : 4; }

int enqueue_group(ldk_plan_s *p, const Group &g, hipStream_t s)
{
    const ldk_batch_desc &D = p->desc;
    unsigned char *ws = static_cast<unsigned char *>(p->ws);
    const bool lat = g.kind == LDK_LATTICE;
    const int64_t n = (int64_t)1 << g.m;
    ldk_pointset ps{};
    ps.kind = g.kind;
    ps.order = LDK_NATURAL;
    ps.R = g.R;
    ps.d = D.d;
    ps.m_max = D.m_max;
    ps.shift = reinterpret_cast<const uint64_t *>(ws + g.ws_shift);
    if (lat) {
        ps.gen = D.lattice_gen;
    } else if (g.ws_cols != (size_t)-1) {
        ps.flags = LDK_GEN_PER_REPLICATION;  // the group's scrambled columns, formed at bind
        ps.gen = reinterpret_cast<const uint64_t *>(ws + g.ws_cols);
    } else {
        ps.gen = D.net_gen;
    }
    ldk_kernel k{};
    k.kind = g.kind;
    k.d = D.d;
    k.alpha = lat ? p->alpha_lat.data() : p->alpha_net.data();
    k.gamma = lat ? D.lattice_kernel.gamma : D.net_kernel.gamma;
    k.zeta = lat ? D.lattice_kernel.zeta : D.net_kernel.zeta;
    void *k1 = ws + g.ws_k1;
    int st = ldk_kernel_column(&k, &ps, nullptr, nullptr, 0, n, D.dtype, k1, s);
    if (st) return st;
    unsigned char *y = static_cast<unsigned char *>(p->y) + g.y_off * esz(D.dtype);
    unsigned char *c = static_cast<unsigned char *>(p->c) + g.y_off * esz(D.dtype);
    return ldk_fit(g.kind, g.R, g.nrhs, g.m, D.dtype, k1, D.sigma2, y, p->lam + g.lam_off, c,
                   p->logdet ? p->logdet + g.ld_off : nullptr, ws + g.ws_fit, s);
}

// The whole table on `s`: groups forked over the plan's streams, joined back.
int enqueue_all(ldk_plan_s *p, hipStream_t s)
{
    const int S = (int)p->streams.size();
    if (S <= 1) {
        for (const Group &g : p->groups) {
            const int st = enqueue_group(p, g, s);
            if (st) return st;
        }
        return LDK_OK;
    }
    LDK_HIP_CHECK(hipEventRecord(p->events[0], s));
    for (int k = 0; k < S; ++k) LDK_HIP_CHECK(hipStreamWaitEvent(p->streams[k], p->events[0], 0));
    // largest groups first, each to the stream with the least work so far
    std::vector<int> order(p->groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    auto work = [&](int i) {
        const Group &g = p->groups[i];
        return (double)g.R * (double)(g.nrhs + 1) * (double)((int64_t)1 << g.m);
    };
    std::sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    std::vector<double> load(S, 0.0);
    for (int i : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[k] += work(i);
        const int st = enqueue_group(p, p->groups[i], p->streams[k]);
        if (st) return st;
    }
    for (int k = 0; k < S; ++k) {
        LDK_HIP_CHECK(hipEventRecord(p->events[1 + k], p->streams[k]));
        LDK_HIP_CHECK(hipStreamWaitEvent(s, p->events[1 + k], 0));
    }
    return LDK_OK;
}

}  // namespace
}  // namespace ldk

using namespace ldk;

extern "C" {

int ldk_plan_create(const ldk_batch_desc *desc, int n_inst, const ldk_instance *inst,
                    ldk_plan *out)
{
    if (!desc || !inst || !out || n_inst < 1) return LDK_EINVAL;
    const ldk_batch_desc &D = *desc;
    if (D.d < 1 || D.d > LDK_MAX_D || D.m_max < 0 || D.m_max > 62) return LDK_EINVAL;
    if (D.dtype != LDK_F64 && D.dtype != LDK_F32) return LDK_EINVAL;
    if (!(D.sigma2 >= 0.0) || D.streams < 1 || D.streams > 8) return LDK_EINVAL;
    bool any_lat = false, any_net = false;
    for (int i = 0; i < n_inst; ++i) {
        const ldk_instance &I = inst[i];
        if (I.kind != LDK_LATTICE && I.kind != LDK_DNET_B2) return LDK_EINVAL;
        if (I.m < 0 || I.m > LDK_MAX_M || I.m > D.m_max || I.nrhs < 1 || !I.shift) return LDK_EINVAL;
        if (I.kind == LDK_LATTICE && I.lms) return LDK_EINVAL;
        (I.kind == LDK_LATTICE ? any_lat : any_net) = true;
    }
    if (any_lat && (!D.lattice_gen || D.lattice_kernel.kind != LDK_LATTICE || D.lattice_kernel.d != D.d ||
                    !D.lattice_kernel.alpha || !D.lattice_kernel.gamma))
        return LDK_EINVAL;
    if (any_net && (!D.net_gen || D.net_kernel.kind != LDK_DNET_B2 || D.net_kernel.d != D.d ||
                    !D.net_kernel.alpha || !D.net_kernel.gamma))
        return LDK_EINVAL;
    ldk_plan_s *p = new ldk_plan_s();
    p->desc = D;
    if (any_lat) p->alpha_lat.assign(D.lattice_kernel.alpha, D.lattice_kernel.alpha + D.d);
    if (any_net) p->alpha_net.assign(D.net_kernel.alpha, D.net_kernel.alpha + D.d);
    p->desc.lattice_kernel.alpha = nullptr;  // the plan keeps its own copies
    p->desc.net_kernel.alpha = nullptr;
    p->inst.assign(inst, inst + n_inst);
    // groups by (kind, m, nrhs, scrambled or not), members in table order
    std::map<std::tuple<int, int, int, int>, int> key_of;
    p->where.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const ldk_instance &I = inst[i];
        const auto key = std::make_tuple(I.kind, I.m, I.nrhs, I.lms ? 1 : 0);
        auto it = key_of.find(key);
        if (it == key_of.end()) {
            it = key_of.emplace(key, (int)p->groups.size()).first;
            Group g{};
            g.kind = I.kind;
            g.m = I.m;
            g.nrhs = I.nrhs;
            p->groups.push_back(g);
        }
        Group &g = p->groups[it->second];
        p->where[i] = {it->second, (int)g.members.size()};
        g.members.push_back(i);
    }
    size_t y = 0, lam = 0, ld = 0, ws = 0;
    for (Group &g : p->groups) {
        g.R = (int)g.members.size();
        if (g.R > 65535) {
            delete p;
            return LDK_ENOTSUP;
        }
        const size_t n = (size_t)1 << g.m;
        g.y_off = y;
        y += (size_t)g.R * g.nrhs * n;
        g.lam_off = lam;
        lam += (size_t)g.R * n;
        g.ld_off = ld;
        ld += (size_t)g.R;
        g.ws_shift = ws;
        ws += al256((size_t)g.R * D.d * 8);
        const bool scr = g.kind == LDK_DNET_B2 && inst[g.members[0]].lms;
        g.ws_lms = (size_t)-1;
        g.ws_cols = (size_t)-1;
        if (scr) {
            g.ws_lms = ws;
            ws += al256((size_t)g.R * D.d * 64 * 8);
            if (D.m_max > 0) {
                g.ws_cols = ws;
                ws += al256((size_t)g.R * D.d * D.m_max * 8);
            }
        }
        g.ws_k1 = ws;
        ws += al256((size_t)g.R * n * esz(D.dtype));
        g.ws_fit = ws;
        g.fit_bytes = ldk_workspace_bytes(LDK_OP_FIT, g.kind, (int64_t)g.R * (g.nrhs + 1), g.m,
                                          D.dtype);
        ws += al256(g.fit_bytes);
    }
    p->arena[LDK_ARENA_Y] = p->arena[LDK_ARENA_C] = y * esz(D.dtype);
    p->arena[LDK_ARENA_LAM] = lam * 8;
    p->arena[LDK_ARENA_LOGDET] = ld * 8;
    p->arena[LDK_ARENA_WS] = ws;
    *out = p;
    return LDK_OK;
}

size_t ldk_plan_arena_bytes(ldk_plan p, int which)
{
    if (!p || which < 0 || which >= LDK_ARENA_COUNT) return 0;
    return p->arena[which];
}

int ldk_plan_instance_offset(ldk_plan p, int i, int which, size_t *offset)
{
    if (!p || !offset || i < 0 || i >= (int)p->inst.size()) return LDK_EINVAL;
    const Group &g = p->groups[p->where[i].first];
    const size_t r = (size_t)p->where[i].second, n = (size_t)1 << g.m;
    switch (which) {
    case LDK_ARENA_Y:
    case LDK_ARENA_C: *offset = g.y_off + r * g.nrhs * n; return LDK_OK;
    case LDK_ARENA_LAM: *offset = g.lam_off + r * n; return LDK_OK;
    case LDK_ARENA_LOGDET: *offset = g.ld_off + r; return LDK_OK;
    case LDK_ARENA_K1: *offset = g.ws_k1 / esz(p->desc.dtype) + r * n; return LDK_OK;
    default: return LDK_EINVAL;
    }
}

int ldk_plan_bind(ldk_plan p, void *y, void *c, double *lam, double *logdet, void *ws,
                  ldk_stream stream)
{
    if (!p || !y || !c || !lam || !ws) return LDK_EINVAL;
    int st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    if (p->exec) {  // a graph captured the previous binding: drop it
        LDK_HIP_CHECK(hipGraphExecDestroy(p->exec));
        LDK_HIP_CHECK(hipGraphDestroy(p->graph));
        p->exec = nullptr;
        p->graph = nullptr;
    }
    p->y = y;
    p->c = c;
    p->lam = lam;
    p->logdet = logdet;
    p->ws = ws;
    const ldk_batch_desc &D = p->desc;
    unsigned char *w8 = static_cast<unsigned char *>(ws);
    for (const Group &g : p->groups) {
        // gather every member's shift (and scrambles) into the group's rows
        for (int r = 0; r < g.R; ++r) {
            const ldk_instance &I = p->inst[g.members[r]];
            LDK_HIP_CHECK(hipMemcpyAsync(w8 + g.ws_shift + (size_t)r * D.d * 8, I.shift,
                                         (size_t)D.d * 8, hipMemcpyDeviceToDevice, s));
            if (g.ws_lms != (size_t)-1)
                LDK_HIP_CHECK(hipMemcpyAsync(w8 + g.ws_lms + (size_t)r * D.d * 64 * 8, I.lms,
                                             (size_t)D.d * 64 * 8, hipMemcpyDeviceToDevice, s));
        }
        if (g.ws_cols != (size_t)-1) {
            // each replication's scrambled columns S_j C_j, once per binding
            // (interlacing of order 1): the column kernel then skips scrambling
            ldk_pointset src{};
            src.kind = LDK_DNET_B2;
            src.order = LDK_NATURAL;
            src.R = g.R;
            src.d = D.d;
            src.m_max = D.m_max;
            src.gen = D.net_gen;
            src.lms = reinterpret_cast<const uint64_t *>(w8 + g.ws_lms);
            st = ldk_interlace(&src, 1, reinterpret_cast<uint64_t *>(w8 + g.ws_cols), stream);
            if (st) return st;
        }
    }
    if (p->streams.empty()) {
        const int S = D.streams;
        p->events.resize(1 + (S > 1 ? S : 0));
        for (auto &e : p->events) LDK_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        if (S > 1) {
            p->streams.resize(S);
            for (auto &q : p->streams) LDK_HIP_CHECK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        }
    }
    p->bound = true;
    return LDK_OK;
}

int ldk_batch_launch(ldk_plan p, ldk_stream stream)
{
    if (!p || !p->bound) return LDK_EINVAL;
    hipStream_t s = as_stream(stream);
    if (p->exec) {
        LDK_HIP_CHECK(hipGraphLaunch(p->exec, s));
        return LDK_OK;
    }
    return enqueue_all(p, s);
}

int ldk_batch_capture(ldk_plan p, ldk_stream stream)
{
    if (!p || !p->bound) return LDK_EINVAL;
    hipStream_t s = as_stream(stream);
    if (!s) return LDK_EINVAL;  // the null stream cannot be captured
    if (p->exec) {
        LDK_HIP_CHECK(hipGraphExecDestroy(p->exec));
        LDK_HIP_CHECK(hipGraphDestroy(p->graph));
        p->exec = nullptr;
        p->graph = nullptr;
    }
    LDK_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const int st = enqueue_all(p, s);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    LDK_HIP_CHECK(e);
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_hip_error(ei);
        return LDK_EDEVICE;
    }
    p->graph = g;
    p->exec = x;
    return LDK_OK;
}

int ldk_plan_stats(ldk_plan p, int *groups, int *kernel_nodes)
{
    if (!p) return LDK_EINVAL;
    if (groups) *groups = (int)p->groups.size();
    if (kernel_nodes) {
        *kernel_nodes = -1;
        if (p->graph) {
            size_t count = 0;
            LDK_HIP_CHECK(hipGraphGetNodes(p->graph, nullptr, &count));
            std::vector<hipGraphNode_t> nodes(count);
            LDK_HIP_CHECK(hipGraphGetNodes(p->graph, nodes.data(), &count));
            int k = 0;
            for (size_t i = 0; i < count; ++i) {
                hipGraphNodeType t;
                LDK_HIP_CHECK(hipGraphNodeGetType(nodes[i], &t));
                k += t == hipGraphNodeTypeKernel;
            }
            *kernel_nodes = k;
        }
    }
    return LDK_OK;
}

int ldk_plan_destroy(ldk_plan p)
{
    if (!p) return LDK_OK;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (auto &q : p->streams) (void)hipStreamDestroy(q);
    for (auto &e : p->events) (void)hipEventDestroy(e);
    delete p;
    return LDK_OK;
}

}  // extern "C"
