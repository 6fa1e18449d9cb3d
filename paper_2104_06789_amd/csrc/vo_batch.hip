// vo_batch.hip -- batches of independent windows (Table 1 per window) over
// concurrent HIP streams.
//
// A window's pose steps are a chain of small, latency-bound launches (one
// workgroup per mean-shift), while its sweeps fill the whole chip.  Windows
// share nothing, so a batch is spread over `lanes` streams, each owning the
// workspace of one context; the hardware queues run the lanes side by side and
// one window's pose chain overlaps the sweeps of the others.  Windows of one
// lane run in stream order and reuse its workspace.  Assignment is
// longest-processing-time first: windows by decreasing cost, each onto the
// lane with the least cost so far.  With VOLDOR_BATCH_GRAPH the whole
// fork/lanes/join sequence is captured into a HIP graph once per distinct call
// and replayed, so the host submits one graph instead of every launch.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "vo_internal.hpp"

using namespace vo;

namespace {

constexpr int kMaxLanes = 16;

// relative cost of a window: its pixel-frames (sweeps, rigidness) plus a
// fixed share per frame for the pose chain (about 0.1 Mpixel-frames of sweep
// time per frame and iteration)
double window_cost(const voldor_window_desc &w)
{
    return (double)w.T * ((double)w.H * (double)w.W + 1.0e5);
}

}  // namespace

struct voldor_batch {
    int lanes;
    int flags;
    int T_max, H_max, W_max, S_max;
    voldor_ctx *ctx[kMaxLanes];
    // lockstep mode: a context per window (windows of a lane are in flight
    // together), the plan of the last call (argument arrays on the device,
    // every lane's windows and steps) and the bytes of that call
    std::vector<voldor_ctx *> wctx;
    unsigned char *plan_dev;
    size_t plan_cap;
    std::vector<std::vector<int>> lane_idx;
    std::vector<std::vector<WinRef>> lane_refs;
    std::vector<std::vector<LockStep>> lane_steps;
    std::vector<unsigned char> plan_key;
    hipStream_t st[kMaxLanes];
    hipEvent_t fork;
    hipEvent_t join[kMaxLanes];
    // graph of the last captured call, with the bytes of that call
    hipGraph_t graph;
    hipGraphExec_t exec;
    std::vector<unsigned char> key;
};

namespace {

void drop_graph(voldor_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->key.clear();
    b->plan_key.clear();   // a plan holds the tuned launch settings of its call
}

// sweep settings of the lanes' first context onto a window context
void copy_tuning(const voldor_ctx *from, voldor_ctx *to)
{
    to->sweep_nt[0] = from->sweep_nt[0];
    to->sweep_nt[1] = from->sweep_nt[1];
    to->sweep_la[0] = from->sweep_la[0];
    to->sweep_la[1] = from->sweep_la[1];
    to->n_sweep_tab = from->n_sweep_tab;
    for (int k = 0; k < from->n_sweep_tab; ++k) to->sweep_tab[k] = from->sweep_tab[k];
}

void assign_lanes(const voldor_window_desc *w, int n, int lanes, std::vector<int> &order,
                  std::vector<int> &lane_of)
{
    order.resize(n);
    lane_of.resize(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return window_cost(w[a]) > window_cost(w[b]); });
    double load[kMaxLanes] = {0};
    for (int i : order) {
        int l = 0;
        for (int k = 1; k < lanes; ++k)
            if (load[k] < load[l]) l = k;
        lane_of[i] = l;
        load[l] += window_cost(w[i]);
    }
}

// fork the lanes off s, enqueue every window on its lane, join them back to s
int batch_enqueue(voldor_batch *b, const voldor_window_desc *w, int n, const voldor_params *p,
                  int32_t *status_out, hipStream_t s)
{
    const int used = std::min(b->lanes, n);
    std::vector<int> order, lane_of;
    assign_lanes(w, n, used, order, lane_of);
    if (hipEventRecord(b->fork, s) != hipSuccess) return VOLDOR_EDEVICE;
    for (int l = 0; l < used; ++l)
        if (hipStreamWaitEvent(b->st[l], b->fork, 0) != hipSuccess) return VOLDOR_EDEVICE;
    int rc = VOLDOR_OK;
    for (int k = 0; k < n && rc == VOLDOR_OK; ++k) {
        const int i = order[k], l = lane_of[i];
        const voldor_window_desc &d = w[i];
        const WindowInit in = {d.init_depth, d.init_rig, d.choice};
        voldor_params pw = *p;
        if (d.n_pose_groups > 0) pw.n_pose_groups = d.n_pose_groups;
        rc = window_enqueue(b->ctx[l], d.flows, d.T, d.H, d.W, d.K, &pw, d.poses, d.depth, d.rigidness,
                            d.loglik, status_out + i, b->st[l], (d.init_depth && d.init_rig) ? &in : nullptr);
    }
    // the join is recorded even after a failed launch, so that s never runs
    // ahead of work that did get enqueued
    for (int l = 0; l < used; ++l) {
        if (hipEventRecord(b->join[l], b->st[l]) != hipSuccess) return VOLDOR_EDEVICE;
        if (hipStreamWaitEvent(s, b->join[l], 0) != hipSuccess) return VOLDOR_EDEVICE;
    }
    return rc;
}

// Lockstep mode: the lanes as above, the windows of each lane advancing
// together (vo_api.hip, lockstep_plan).  The plan of a call is built on the
// host and uploaded before anything is enqueued; it is kept, with the call's
// bytes, for the next call with the same bytes (a captured graph reads it).
int lockstep_prepare(voldor_batch *b, const voldor_window_desc *w, int n, const voldor_params *p,
                     const std::vector<unsigned char> &key, hipStream_t s)
{
    if (!b->plan_key.empty() && key == b->plan_key) return VOLDOR_OK;
    // nothing enqueued before may still read the plan buffer or use the contexts
    if (hipStreamSynchronize(s) != hipSuccess) return VOLDOR_EDEVICE;
    for (int l = 0; l < b->lanes; ++l)
        if (hipStreamSynchronize(b->st[l]) != hipSuccess) return VOLDOR_EDEVICE;
    drop_graph(b);   // a captured graph reads the plan buffer rewritten below
    while ((int)b->wctx.size() < n) {
        voldor_ctx *c = nullptr;
        const int rc = voldor_create(&c, b->T_max, b->H_max, b->W_max, b->S_max);
        if (rc) return rc;
        b->wctx.push_back(c);
    }
    for (int i = 0; i < n; ++i) copy_tuning(b->ctx[0], b->wctx[i]);
    const int used = std::min(b->lanes, n);
    std::vector<int> order, lane_of;
    assign_lanes(w, n, used, order, lane_of);
    b->lane_idx.assign(used, std::vector<int>());
    for (int k = 0; k < n; ++k) b->lane_idx[lane_of[order[k]]].push_back(order[k]);
    b->lane_refs.assign(used, std::vector<WinRef>());
    b->lane_steps.assign(used, std::vector<LockStep>());
    Plan plan;
    for (int l = 0; l < used; ++l) {
        std::vector<voldor_ctx *> wc;
        for (int i : b->lane_idx[l]) wc.push_back(b->wctx[i]);
        lockstep_plan(wc.data(), w, b->lane_idx[l], p, plan, b->lane_refs[l], b->lane_steps[l]);
    }
    if (plan.host.size() > b->plan_cap) {
        if (b->plan_dev) (void)hipFree(b->plan_dev);
        b->plan_dev = nullptr;
        b->plan_cap = 0;
        if (hipMalloc((void **)&b->plan_dev, plan.host.size()) != hipSuccess) return VOLDOR_ENOMEM;
        b->plan_cap = plan.host.size();
    }
    if (!plan.host.empty() &&
        hipMemcpy(b->plan_dev, plan.host.data(), plan.host.size(), hipMemcpyHostToDevice) != hipSuccess)
        return VOLDOR_EDEVICE;
    b->plan_key = key;
    return VOLDOR_OK;
}

int lockstep_enqueue(voldor_batch *b, const voldor_window_desc *w, const voldor_params *p,
                     int32_t *status_out, hipStream_t s)
{
    const int used = (int)b->lane_idx.size();
    if (hipEventRecord(b->fork, s) != hipSuccess) return VOLDOR_EDEVICE;
    for (int l = 0; l < used; ++l)
        if (hipStreamWaitEvent(b->st[l], b->fork, 0) != hipSuccess) return VOLDOR_EDEVICE;
    int rc = VOLDOR_OK;
    for (int l = 0; l < used && rc == VOLDOR_OK; ++l)
        rc = lockstep_run(b->ctx[l], b->lane_refs[l], b->lane_steps[l], w, b->lane_idx[l], p, b->plan_dev,
                          status_out, b->st[l]);
    for (int l = 0; l < used; ++l) {
        if (hipEventRecord(b->join[l], b->st[l]) != hipSuccess) return VOLDOR_EDEVICE;
        if (hipStreamWaitEvent(s, b->join[l], 0) != hipSuccess) return VOLDOR_EDEVICE;
    }
    return rc;
}

void call_key(const voldor_window_desc *w, int n, const voldor_params *p, const int32_t *status_out,
              hipStream_t s, std::vector<unsigned char> &key)
{
    key.clear();
    auto put = [&](const void *v, size_t bytes) {
        const unsigned char *c = (const unsigned char *)v;
        key.insert(key.end(), c, c + bytes);
    };
    put(&n, sizeof n);
    put(&status_out, sizeof status_out);
    put(&s, sizeof s);
    put(p, sizeof *p);
    put(w, sizeof(voldor_window_desc) * (size_t)n);
}

}  // namespace

extern "C" {

int voldor_batch_create(voldor_batch **out, int lanes, int T_max, int H_max, int W_max, int S_max,
                        int flags)
{
    if (!out) return VOLDOR_EINVAL;
    *out = nullptr;
    if (lanes < 1 || lanes > kMaxLanes || (flags & ~(VOLDOR_BATCH_GRAPH | VOLDOR_BATCH_LOCKSTEP)) != 0)
        return VOLDOR_EINVAL;
    voldor_batch *b = new (std::nothrow) voldor_batch();
    if (!b) return VOLDOR_ENOMEM;
    b->lanes = lanes;
    b->flags = flags;
    b->T_max = T_max;
    b->H_max = H_max;
    b->W_max = W_max;
    b->S_max = S_max;
    int rc = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
    for (int l = 0; l < lanes && rc == VOLDOR_OK; ++l) {
        rc = voldor_create(&b->ctx[l], T_max, H_max, W_max, S_max);
        if (rc == VOLDOR_OK && hipStreamCreateWithFlags(&b->st[l], hipStreamNonBlocking) != hipSuccess)
            rc = VOLDOR_EDEVICE;
        if (rc == VOLDOR_OK && hipEventCreateWithFlags(&b->join[l], hipEventDisableTiming) != hipSuccess)
            rc = VOLDOR_EDEVICE;
    }
    if (rc != VOLDOR_OK) {
        voldor_batch_destroy(b);
        return rc;
    }
    *out = b;
    return VOLDOR_OK;
}

int voldor_batch_set_sweep_threads(voldor_batch *b, int rows, int cols)
{
    if (!b) return VOLDOR_EINVAL;
    for (int l = 0; l < b->lanes; ++l) {
        const int rc = voldor_set_sweep_threads(b->ctx[l], rows, cols);
        if (rc) return rc;
    }
    drop_graph(b);   // a captured graph holds the old launches
    return VOLDOR_OK;
}

int voldor_batch_set_sweep_lookahead(voldor_batch *b, int rows, int cols)
{
    if (!b) return VOLDOR_EINVAL;
    for (int l = 0; l < b->lanes; ++l) {
        const int rc = voldor_set_sweep_lookahead(b->ctx[l], rows, cols);
        if (rc) return rc;
    }
    drop_graph(b);   // a captured graph holds the old launches
    return VOLDOR_OK;
}

int voldor_batch_autotune(voldor_batch *b, const voldor_window_desc *wins, int n, const voldor_params *p,
                          void *stream)
{
    if (!b || !wins || n < 1 || !p) return VOLDOR_EINVAL;
    for (int i = 0; i < n; ++i) {
        bool seen = false;
        for (int k = 0; k < i && !seen; ++k)
            seen = wins[k].T == wins[i].T && wins[k].H == wins[i].H && wins[k].W == wins[i].W;
        if (seen) continue;
        const voldor_window_desc &d = wins[i];
        const int rc = voldor_autotune(b->ctx[0], d.flows, d.T, d.H, d.W, d.K, p, nullptr, nullptr, stream);
        if (rc) return rc;
    }
    for (int l = 1; l < b->lanes; ++l) {
        voldor_ctx *c = b->ctx[l];
        c->n_sweep_tab = b->ctx[0]->n_sweep_tab;
        for (int k = 0; k < c->n_sweep_tab; ++k) c->sweep_tab[k] = b->ctx[0]->sweep_tab[k];
    }
    drop_graph(b);   // a captured graph holds the old launches
    return VOLDOR_OK;
}

int voldor_batch_set_timing(voldor_batch *b, int enable)
{
    if (!b) return VOLDOR_EINVAL;
    for (int l = 0; l < b->lanes; ++l) {
        const int rc = voldor_set_timing(b->ctx[l], enable);
        if (rc) return rc;
    }
    drop_graph(b);   // a captured graph holds (or lacks) the event records
    return VOLDOR_OK;
}

int voldor_batch_timing_summary(voldor_batch *b, double *out, int *n_windows)
{
    if (!b || !out) return VOLDOR_EINVAL;
    for (int i = 0; i < 8; ++i) out[i] = 0.0;
    // out[7]: the time during which at least one lane ran sweeps, from the
    // sweep intervals of every recorded window (the real-time counter is one
    // clock for the whole device, so intervals of different lanes compare)
    std::vector<std::pair<unsigned long long, unsigned long long>> iv;
    double khz = 0.0;
    for (int l = 0; l < b->lanes; ++l) {
        voldor_ctx *c = b->ctx[l];
        if (!c->timing) return VOLDOR_EINVAL;
        if (c->tw_count == 0) continue;
        if (hipStreamSynchronize(c->last_stream) != hipSuccess ||
            hipMemcpy(c->stamps_host, c->stamps, sizeof(unsigned long long) * kTimingRing * kEvPerWin,
                      hipMemcpyDeviceToHost) != hipSuccess)
            return VOLDOR_EDEVICE;
        khz = c->stamp_khz;
        const long long n = c->tw_count < kTimingRing ? c->tw_count : kTimingRing;
        for (long long k = c->tw_count - n; k < c->tw_count; ++k) {
            const int w = (int)(k % kTimingRing);
            const unsigned long long *st = c->stamps_host + w * kEvPerWin;
            for (int i = 1; i < c->ev_n[w]; ++i)
                if (c->ev_phase[w][i] == kPhaseSweep && st[i] > st[i - 1]) iv.emplace_back(st[i - 1], st[i]);
        }
    }
    std::sort(iv.begin(), iv.end());
    unsigned long long covered = 0, lo = 0, hi = 0;
    bool open = false;
    for (const auto &x : iv) {
        if (open && x.first <= hi) {
            if (x.second > hi) hi = x.second;
        } else {
            if (open) covered += hi - lo;
            lo = x.first;
            hi = x.second;
            open = true;
        }
    }
    if (open) covered += hi - lo;
    const double union_ms = khz > 0.0 ? (double)covered / khz : 0.0;
    int total = 0;
    for (int l = 0; l < b->lanes; ++l) {
        double m[8];
        int n = 0;
        const int rc = voldor_timing_summary(b->ctx[l], m, &n);
        if (rc) return rc;
        for (int i = 0; i < 7; ++i) out[i] += m[i] * n;
        total += n;
    }
    out[7] = union_ms;
    if (n_windows) *n_windows = total;
    return VOLDOR_OK;
}

void voldor_batch_destroy(voldor_batch *b)
{
    if (!b) return;
    for (int l = 0; l < b->lanes; ++l)
        if (b->st[l]) (void)hipStreamSynchronize(b->st[l]);
    drop_graph(b);
    for (int l = 0; l < b->lanes; ++l) {
        if (b->join[l]) (void)hipEventDestroy(b->join[l]);
        if (b->st[l]) (void)hipStreamDestroy(b->st[l]);
        voldor_destroy(b->ctx[l]);
    }
    for (voldor_ctx *c : b->wctx) voldor_destroy(c);
    if (b->plan_dev) (void)hipFree(b->plan_dev);
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
}

int voldor_window_batch(voldor_batch *b, const voldor_window_desc *wins, int n, const voldor_params *p,
                        int32_t *status_out, void *stream)
{
    if (!b || !wins || n < 1 || !status_out || ((uintptr_t)status_out & 3) != 0) return VOLDOR_EINVAL;
    if (!p) return VOLDOR_EINVAL;
    for (int i = 0; i < n; ++i) {
        const voldor_window_desc &d = wins[i];
        if (d.n_pose_groups < 0) return VOLDOR_EINVAL;
        voldor_params pw = *p;
        if (d.n_pose_groups > 0) pw.n_pose_groups = d.n_pose_groups;
        if (!window_args_ok(b->ctx[0], d.flows, d.T, d.H, d.W, d.K, &pw, d.poses, d.depth, d.rigidness))
            return VOLDOR_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool lock = (b->flags & VOLDOR_BATCH_LOCKSTEP) != 0;
    if (lock) {
        // lockstep windows start from their own bootstrap with the KDE pose start
        if (p->pose_start != 0) return VOLDOR_EINVAL;
        for (int i = 0; i < n; ++i)
            if (wins[i].init_depth || wins[i].init_rig) return VOLDOR_EINVAL;
    }
    const bool graph = (b->flags & VOLDOR_BATCH_GRAPH) && s != nullptr;
    std::vector<unsigned char> key;
    if (lock || graph) call_key(wins, n, p, status_out, s, key);
    if (graph && b->exec && key == b->key)
        return hipGraphLaunch(b->exec, s) == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
    if (graph) drop_graph(b);
    if (lock) {
        const int rc = lockstep_prepare(b, wins, n, p, key, s);
        if (rc) return rc;
    }
    if (!graph)
        return lock ? lockstep_enqueue(b, wins, p, status_out, s) : batch_enqueue(b, wins, n, p, status_out, s);

    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return VOLDOR_EDEVICE;
    const int rc = lock ? lockstep_enqueue(b, wins, p, status_out, s) : batch_enqueue(b, wins, n, p, status_out, s);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (rc != VOLDOR_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc != VOLDOR_OK ? rc : VOLDOR_EDEVICE;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return VOLDOR_EDEVICE;
    }
    b->graph = g;
    b->exec = ex;
    b->key.swap(key);
    return hipGraphLaunch(b->exec, s) == hipSuccess ? VOLDOR_OK : VOLDOR_EDEVICE;
}

}  // extern "C"
