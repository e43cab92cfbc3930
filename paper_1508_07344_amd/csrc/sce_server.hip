// Host runtime of the batched serving API (sce_server_*): request queue,
// first-in first-out admission by device footprint into one arena, slot and
// work-list management, the tick loop, retirement and latency statistics.
// The arithmetic of every pass runs in kernels_serve.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "sce.h"
#include "sce_serve.h"

using sce::ReqDesc;
using sce::ServeItem;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t id = 0;
    ReqDesc d{};            // offsets relative to the request's base until admitted
    size_t bytes = 0;
    double self_w = 0.0;    // (sum q^2 / (eps0 V)) sum_H S^2 / |k|^2
    std::vector<double> x, v, q, m;
    double t_submit = 0.0;
    double t_admit = 0.0;
    size_t base = 0;
    int slot = -1;
    int64_t pass = 0;       // host mirror of the device pass counter
};

struct Result {
    std::vector<double> x, v, F;  // [dim][N]
    double diag[sce::kServeDiag];
    double self_w = 0.0, dt = 0.0;
    int64_t n_steps = 0;
    int dim = 3;
};

// First-fit allocator over the arena, free blocks kept sorted by offset.
struct Arena {
    std::map<size_t, size_t> free_;
    size_t used = 0, peak = 0;
    void reset(size_t bytes)
    {
        free_.clear();
        free_[0] = bytes;
        used = peak = 0;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used += bytes;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        used -= bytes;
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
};

// A device buffer with a pinned host mirror, grown on demand (only between ticks,
// when the stream is idle).
template <typename E>
struct Mirrored {
    E *dev = nullptr, *host = nullptr;
    size_t cap = 0;
    hipError_t reserve(size_t n)
    {
        if (n <= cap) return hipSuccess;
        size_t c = std::max<size_t>(n, cap * 2);
        c = std::max<size_t>(c, 256);
        if (dev) (void)hipFree(dev);
        if (host) (void)hipHostFree(host);
        dev = nullptr;
        host = nullptr;
        cap = 0;
        hipError_t e = hipMalloc(&dev, c * sizeof(E));
        if (e != hipSuccess) return e;
        e = hipHostMalloc(&host, c * sizeof(E), hipHostMallocDefault);
        if (e != hipSuccess) return e;
        cap = c;
        return hipSuccess;
    }
    void release()
    {
        if (dev) (void)hipFree(dev);
        if (host) (void)hipHostFree(host);
        dev = host = nullptr;
        cap = 0;
    }
};

int64_t half_modes(int n, int dim)
{
    const int64_t M = 2 * n + 1;
    return dim == 2 ? (M * M - 1) / 2 : (M * M * M - 1) / 2;
}

double shape_host(int kind, double a, double kx, double ky, double kz)
{
    if (kind == SCE_SHAPE_GAUSSIAN) return std::exp(-0.5 * (kx * kx + ky * ky + kz * kz) * a * a);
    if (kind == SCE_SHAPE_TENT) {
        double s = 1.0;
        for (double k : {kx, ky, kz}) {
            const double u = 0.5 * k * a;
            const double sc = u == 0.0 ? 1.0 : std::sin(u) / u;
            s *= sc * sc;
        }
        return s;
    }
    return 1.0;
}

}  // namespace

struct sce_server_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool broken = false;
    int prec = SCE_PREC_FP32;
    int elem = 4;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    Arena alloc;
    int max_slots = 0;
    std::vector<int> free_slots;
    Mirrored<ReqDesc> desc;
    Mirrored<ServeItem> dep, red, frc;
    Mirrored<int> slots;
    Mirrored<int> counts;    // ndep, nred, nfrc, nslots on the device
    Mirrored<double> stage;  // retirement staging
    int ndep = 0, nred = 0, nfrc = 0, nslots = 0;
    bool dirty = true;
    // the tick's launches captured once per work list and replayed
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    size_t gcap[4] = {0, 0, 0, 0};  // list capacities the graph was captured with

    uint64_t next_id = 1;
    std::deque<std::unique_ptr<Request>> queue;
    std::vector<std::unique_ptr<Request>> active;
    std::unordered_map<uint64_t, Result> done;
    std::deque<uint64_t> unpolled;
    // sum_H S^2/|k|^2 per (n_max, shape, a, L)
    std::map<std::tuple<int, int, double, double, int>, double> self_cache;

    // statistics
    std::vector<std::pair<double, int>> tick_lat;  // (seconds, resident requests)
    std::vector<std::pair<double, int>> tick_gpu;  // device time of the tick's kernels
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    std::vector<double> waits;
    int64_t ticks = 0, request_steps = 0, requests_done = 0;
    double busy = 0.0, pairs = 0.0;

    std::string err;
};

namespace {

sce_status sfail(sce_server s, sce_status st, const std::string &msg)
{
    if (s) s->err = msg;
    return st;
}

sce_status shipfail(sce_server s, hipError_t e, const char *what)
{
    if (s) {
        s->broken = true;
        s->err = std::string(what) + ": " + hipGetErrorString(e);
    }
    return SCE_EDEVICE;
}

#define SHIP(s, expr)                                        \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return shipfail(s, _e, #expr); \
    } while (0)

// sum over the stored modes of S^2 / |k|^2 (dim 2: the n_x = 0 slice)
double self_sum(sce_server s, int n, int kind, double a, double L, int dim)
{
    const auto key = std::make_tuple(n, kind, a, L, dim);
    auto it = s->self_cache.find(key);
    if (it != s->self_cache.end()) return it->second;
    const double f = 6.283185307179586476925286766559 / L;
    double sum = 0.0;
    for (int nx = 0; nx <= (dim == 2 ? 0 : n); ++nx)
        for (int ny = -n; ny <= n; ++ny)
            for (int nz = -n; nz <= n; ++nz) {
                const bool inh = nx > 0 || (nx == 0 && (ny > 0 || (ny == 0 && nz > 0)));
                if (!inh) continue;
                const double kx = f * nx, ky = f * ny, kz = f * nz;
                const double S = shape_host(kind, a, kx, ky, kz);
                sum += S * S / (kx * kx + ky * ky + kz * kz);
            }
    s->self_cache[key] = sum;
    return sum;
}

sce_status admit(sce_server s, double t0)
{
    while (!s->queue.empty() && !s->free_slots.empty()) {
        Request &r = *s->queue.front();
        size_t base;
        if (!s->alloc.alloc(r.bytes, base)) break;
        const int slot = s->free_slots.back();
        s->free_slots.pop_back();
        r.base = base;
        r.slot = slot;
        r.t_admit = t0;
        ReqDesc d = r.d;
        for (int64_t *o : {&d.o_pos, &d.o_vel, &d.o_q, &d.o_m, &d.o_F, &d.o_part, &d.o_ftab,
                           &d.o_psi0, &d.o_rpart, &d.o_fpart, &d.o_diag})
            *o += (int64_t)base;
        const size_t N = (size_t)d.N;
        char *b = s->arena;
        SHIP(s, hipMemcpyAsync(b + d.o_pos, r.x.data(), 24 * N, hipMemcpyHostToDevice, s->stream));
        SHIP(s, hipMemcpyAsync(b + d.o_vel, r.v.data(), 24 * N, hipMemcpyHostToDevice, s->stream));
        SHIP(s, hipMemcpyAsync(b + d.o_q, r.q.data(), 8 * N, hipMemcpyHostToDevice, s->stream));
        SHIP(s, hipMemcpyAsync(b + d.o_m, r.m.data(), 8 * N, hipMemcpyHostToDevice, s->stream));
        s->desc.host[slot] = d;
        SHIP(s, hipMemcpyAsync(s->desc.dev + slot, s->desc.host + slot, sizeof(ReqDesc),
                               hipMemcpyHostToDevice, s->stream));
        s->waits.push_back(t0 - r.t_submit);
        s->active.push_back(std::move(s->queue.front()));
        s->queue.pop_front();
        s->dirty = true;
    }
    return SCE_OK;
}

sce_status build_lists(sce_server s)
{
    // most expensive requests first, so their blocks start early in each launch
    std::vector<Request *> order;
    for (auto &r : s->active) order.push_back(r.get());
    std::stable_sort(order.begin(), order.end(), [](const Request *a, const Request *b) {
        return std::make_pair(a->d.n, a->d.N) > std::make_pair(b->d.n, b->d.N);
    });
    size_t nd = 0, nr = 0, nf = 0;
    for (Request *r : order) {
        nd += (size_t)(r->d.Rp / 64) * r->d.segs;
        nr += r->d.rblocks;
        nf += r->d.fblocks;
    }
    SHIP(s, s->dep.reserve(nd));
    SHIP(s, s->red.reserve(nr));
    SHIP(s, s->frc.reserve(nf));
    SHIP(s, s->slots.reserve(order.size()));
    size_t id = 0, ir = 0, jf = 0, is = 0;
    for (Request *r : order) {
        const int tiles = r->d.Rp / 64;
        for (int i = 0; i < tiles * r->d.segs; ++i) s->dep.host[id++] = ServeItem{r->slot, i};
        for (int i = 0; i < r->d.rblocks; ++i) s->red.host[ir++] = ServeItem{r->slot, i};
        for (int i = 0; i < r->d.fblocks; ++i) s->frc.host[jf++] = ServeItem{r->slot, i};
        s->slots.host[is++] = r->slot;
    }
    s->ndep = (int)nd;
    s->nred = (int)nr;
    s->nfrc = (int)nf;
    s->nslots = (int)order.size();
    if (nd)
        SHIP(s, hipMemcpyAsync(s->dep.dev, s->dep.host, nd * sizeof(ServeItem), hipMemcpyHostToDevice, s->stream));
    if (nr)
        SHIP(s, hipMemcpyAsync(s->red.dev, s->red.host, nr * sizeof(ServeItem), hipMemcpyHostToDevice, s->stream));
    if (nf)
        SHIP(s, hipMemcpyAsync(s->frc.dev, s->frc.host, nf * sizeof(ServeItem), hipMemcpyHostToDevice, s->stream));
    if (is)
        SHIP(s, hipMemcpyAsync(s->slots.dev, s->slots.host, is * sizeof(int), hipMemcpyHostToDevice, s->stream));
    SHIP(s, s->counts.reserve(4));
    s->counts.host[0] = s->ndep;
    s->counts.host[1] = s->nred;
    s->counts.host[2] = s->nfrc;
    s->counts.host[3] = s->nslots;
    SHIP(s, hipMemcpyAsync(s->counts.dev, s->counts.host, 4 * sizeof(int), hipMemcpyHostToDevice, s->stream));
    s->dirty = false;
    return SCE_OK;
}

void drop_graph(sce_server s)
{
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->gexec = nullptr;
    s->graph = nullptr;
}

// Launch one tick's kernels: replayed from a HIP graph whose grids cover the
// work lists' capacities (blocks beyond the device-side counts return at
// once), captured again only when a capacity grows; or launched directly with
// exact grids.
sce_status launch_tick(sce_server s)
{
    if (!s->use_graph) {
        const hipError_t e = sce::launch_serve_tick(s->stream, s->elem, s->desc.dev, s->arena, s->dep.dev,
                                                    s->ndep, s->red.dev, s->nred, s->frc.dev, s->nfrc,
                                                    s->slots.dev, s->nslots, s->counts.dev);
        return e == hipSuccess ? SCE_OK : shipfail(s, e, "launch_serve_tick");
    }
    const size_t cap[4] = {s->dep.cap, s->red.cap, s->frc.cap, s->slots.cap};
    if (!s->gexec || std::memcmp(cap, s->gcap, sizeof(cap)) != 0) {
        drop_graph(s);
        SHIP(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
        const hipError_t le = sce::launch_serve_tick(s->stream, s->elem, s->desc.dev, s->arena, s->dep.dev,
                                                     (int)cap[0], s->red.dev, (int)cap[1], s->frc.dev,
                                                     (int)cap[2], s->slots.dev, (int)cap[3], s->counts.dev);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(s->stream, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return shipfail(s, le, "launch_serve_tick (capture)");
        }
        SHIP(s, ce);
        s->graph = g;
        SHIP(s, hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0));
        std::memcpy(s->gcap, cap, sizeof(cap));
    }
    SHIP(s, hipGraphLaunch(s->gexec, s->stream));
    return SCE_OK;
}

// Requests whose last pass runs in this tick: enqueue the copies of their
// final state behind the tick's kernels (one synchronisation covers both).
sce_status stage_finishing(sce_server s, std::vector<Request *> &fin)
{
    fin.clear();
    for (auto &r : s->active)
        if (r->pass == r->d.n_steps) fin.push_back(r.get());
    if (fin.empty()) return SCE_OK;
    size_t tot = 0;
    for (Request *r : fin) tot += 9 * (size_t)r->d.N + sce::kServeDiag;
    SHIP(s, s->stage.reserve(tot));
    return SCE_OK;
}

sce_status copy_finishing(sce_server s, const std::vector<Request *> &fin)
{
    size_t off = 0;
    for (Request *r : fin) {
        const ReqDesc &d = s->desc.host[r->slot];
        const size_t N = (size_t)d.N;
        double *h = s->stage.host + off;
        SHIP(s, hipMemcpyAsync(h, s->arena + d.o_pos, 24 * N, hipMemcpyDeviceToHost, s->stream));
        SHIP(s, hipMemcpyAsync(h + 3 * N, s->arena + d.o_vel, 24 * N, hipMemcpyDeviceToHost, s->stream));
        SHIP(s, hipMemcpyAsync(h + 6 * N, s->arena + d.o_F, 24 * N, hipMemcpyDeviceToHost, s->stream));
        SHIP(s, hipMemcpyAsync(h + 9 * N, s->arena + d.o_diag, 8 * sce::kServeDiag,
                               hipMemcpyDeviceToHost, s->stream));
        off += 9 * N + sce::kServeDiag;
    }
    return SCE_OK;
}

// After the tick's synchronisation: move the staged results to host storage
// and release the finished requests' arena blocks and slots.
void retire(sce_server s, const std::vector<Request *> &fin)
{
    if (fin.empty()) return;
    size_t off = 0;
    for (Request *r : fin) {
        const size_t N = (size_t)r->d.N;
        const double *h = s->stage.host + off;
        Result res;
        // a two-dimensional request's vectors are the stored (y, z) components
        const size_t o = r->d.dim == 2 ? N : 0;
        res.dim = r->d.dim;
        res.x.assign(h + o, h + 3 * N);
        res.v.assign(h + 3 * N + o, h + 6 * N);
        res.F.assign(h + 6 * N + o, h + 9 * N);
        std::memcpy(res.diag, h + 9 * N, sizeof(res.diag));
        res.self_w = r->self_w;
        res.dt = r->d.dt;
        res.n_steps = r->d.n_steps;
        off += 9 * N + sce::kServeDiag;
        s->done.emplace(r->id, std::move(res));
        s->unpolled.push_back(r->id);
        s->alloc.release(r->base, r->bytes);
        s->free_slots.push_back(r->slot);
        ++s->requests_done;
    }
    s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                   [](const std::unique_ptr<Request> &r) { return r->pass > r->d.n_steps; }),
                    s->active.end());
    s->dirty = true;
}

void fill_diag(sce_diag *o, const double *d, double self_w, int64_t step, double dt, int dim)
{
    o->step = step;
    o->time = (double)step * dt;
    o->kinetic = d[0];
    o->field = d[1];
    o->field_self = self_w;
    o->interaction = d[2];
    o->total = d[0] + d[1];
    o->momentum[0] = dim == 2 ? d[4] : d[3];
    o->momentum[1] = dim == 2 ? d[5] : d[4];
    o->momentum[2] = dim == 2 ? 0.0 : d[5];
    o->momentum_abs_sum = d[6];
    o->rho_abs_max = d[7];
}

double weighted_pct(std::vector<std::pair<double, int>> v, double p)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    double tot = 0.0;
    for (auto &e : v) tot += e.second;
    double acc = 0.0;
    for (auto &e : v) {
        acc += e.second;
        if (acc >= p * tot) return e.first;
    }
    return v.back().first;
}

}  // namespace

extern "C" {

sce_status sce_server_create(const sce_server_opts *opts, sce_server *out)
{
    if (!out) return SCE_EINVAL;
    *out = nullptr;
    sce_server_opts o{};
    if (opts) o = *opts;
    if (o.max_active < 0) return SCE_EINVAL;
    if (o.precision != SCE_PREC_FP32 && o.precision != SCE_PREC_FP64) return SCE_ENOTSUP;
    sce_server s = new (std::nothrow) sce_server_s;
    if (!s) return SCE_ENOMEM;
    s->prec = o.precision;
    s->elem = o.precision == SCE_PREC_FP64 ? 8 : 4;
    s->arena_bytes = o.hbm_budget_bytes ? o.hbm_budget_bytes : ((size_t)4 << 30);
    s->max_slots = o.max_active ? o.max_active : 4096;
    s->use_graph = o.no_graph == 0;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) {
        if (o.hip_stream) {
            s->stream = (hipStream_t)o.hip_stream;
        } else {
            e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
            s->own_stream = e == hipSuccess;
        }
    }
    if (e == hipSuccess) e = hipEventCreate(&s->ev_a);
    if (e == hipSuccess) e = hipEventCreate(&s->ev_b);
    if (e == hipSuccess) e = hipMalloc(&s->arena, s->arena_bytes);
    if (e == hipSuccess) e = s->desc.reserve((size_t)s->max_slots);
    if (e != hipSuccess) {
        sce_server_destroy(s);
        return e == hipErrorOutOfMemory ? SCE_ENOMEM : SCE_EDEVICE;
    }
    std::memset(s->desc.host, 0, sizeof(ReqDesc) * s->max_slots);
    s->alloc.reset(s->arena_bytes);
    for (int i = s->max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    *out = s;
    return SCE_OK;
}

sce_status sce_server_submit(sce_server s, const sce_request *r, uint64_t *id)
{
    if (!s || !r || !id) return sfail(s, SCE_EINVAL, "null argument");
    if (s->broken) return sfail(s, SCE_EDEVICE, "server unusable after a device error");
    if (!(r->L > 0.0) || !std::isfinite(r->L)) return sfail(s, SCE_EINVAL, "L must be finite and > 0");
    if (r->n_max < 1 || r->n_max > sce::kServeMaxN)
        return sfail(s, SCE_EINVAL, "n_max must be in 1..16 for served requests");
    if (r->shape_kind < SCE_SHAPE_DELTA || r->shape_kind > SCE_SHAPE_TENT)
        return sfail(s, SCE_EINVAL, "unknown shape kind");
    if (!(r->a >= 0.0) || !std::isfinite(r->a)) return sfail(s, SCE_EINVAL, "shape width must be >= 0");
    if (!(r->eps0 > 0.0) || !std::isfinite(r->eps0)) return sfail(s, SCE_EINVAL, "eps0 must be > 0");
    if (!std::isfinite(r->dt)) return sfail(s, SCE_EINVAL, "dt must be finite");
    if (r->N < 1 || r->N > ((int64_t)1 << 31)) return sfail(s, SCE_EINVAL, "N out of range");
    if (r->n_steps < 0) return sfail(s, SCE_EINVAL, "n_steps must be >= 0");
    if (r->dim != 0 && r->dim != 2 && r->dim != 3) return sfail(s, SCE_EINVAL, "dim must be 2 or 3");
    const int dim = r->dim == 2 ? 2 : 3;
    if (!r->x || !r->v || !r->q || !r->m) return sfail(s, SCE_EINVAL, "null particle array");
    for (int64_t j = 0; j < r->N; ++j)
        if (!(r->m[j] > 0.0)) return sfail(s, SCE_EINVAL, "masses must be > 0");
    auto q = std::make_unique<Request>();
    ReqDesc &d = q->d;
    d.N = r->N;
    d.n = r->n_max;
    d.shape = r->shape_kind;
    d.dim = dim;
    d.L = r->L;
    d.invL = 1.0 / r->L;
    d.a = r->a;
    d.eps0 = r->eps0;
    d.dt = r->dt;
    d.pass = 0;
    d.n_steps = r->n_steps;
    q->bytes = sce::serve_layout(d, s->elem);
    if (q->bytes > s->arena_bytes)
        return sfail(s, SCE_EINVAL, "request footprint exceeds the server's device budget");
    const size_t N = (size_t)r->N;
    if (dim == 2) {
        // stored as (0, x, y)
        q->x.assign(3 * N, 0.0);
        q->v.assign(3 * N, 0.0);
        std::memcpy(q->x.data() + N, r->x, 2 * N * sizeof(double));
        std::memcpy(q->v.data() + N, r->v, 2 * N * sizeof(double));
    } else {
        q->x.assign(r->x, r->x + 3 * N);
        q->v.assign(r->v, r->v + 3 * N);
    }
    q->q.assign(r->q, r->q + N);
    q->m.assign(r->m, r->m + N);
    double q2 = 0.0;
    for (size_t j = 0; j < N; ++j) q2 += r->q[j] * r->q[j];
    const double meas = dim == 2 ? r->L * r->L : r->L * r->L * r->L;
    q->self_w = q2 / (r->eps0 * meas) * self_sum(s, r->n_max, r->shape_kind, r->a, r->L, dim);
    q->id = s->next_id++;
    q->t_submit = now_s();
    *id = q->id;
    s->queue.push_back(std::move(q));
    return SCE_OK;
}

sce_status sce_server_tick(sce_server s, int32_t *n_active, int32_t *n_queued)
{
    if (!s) return SCE_EINVAL;
    if (s->broken) return sfail(s, SCE_EDEVICE, "server unusable after a device error");
    SHIP(s, hipSetDevice(s->device));
    const double t0 = now_s();
    sce_status st = admit(s, t0);
    if (st != SCE_OK) return st;
    if (s->dirty) {
        st = build_lists(s);
        if (st != SCE_OK) return st;
    }
    if (!s->active.empty()) {
        std::vector<Request *> fin;
        st = stage_finishing(s, fin);
        if (st != SCE_OK) return st;
        SHIP(s, hipEventRecord(s->ev_a, s->stream));
        st = launch_tick(s);
        if (st != SCE_OK) return st;
        SHIP(s, hipEventRecord(s->ev_b, s->stream));
        st = copy_finishing(s, fin);
        if (st != SCE_OK) return st;
        SHIP(s, hipStreamSynchronize(s->stream));
        float gpu_ms = 0.f;
        SHIP(s, hipEventElapsedTime(&gpu_ms, s->ev_a, s->ev_b));
        const int na = (int)s->active.size();
        double pr = 0.0;
        for (auto &r : s->active) {
            ++r->pass;
            pr += (double)r->d.N * (double)half_modes(r->d.n, r->d.dim);
            if (!r->x.empty()) {  // uploaded at admission; the copies have completed
                std::vector<double>().swap(r->x);
                std::vector<double>().swap(r->v);
                std::vector<double>().swap(r->q);
                std::vector<double>().swap(r->m);
            }
        }
        retire(s, fin);
        const double dt = now_s() - t0;
        s->tick_lat.emplace_back(dt, na);
        s->tick_gpu.emplace_back(1e-3 * (double)gpu_ms, na);
        ++s->ticks;
        s->request_steps += na;
        s->busy += dt;
        s->pairs += pr;
    }
    if (n_active) *n_active = (int32_t)s->active.size();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return SCE_OK;
}

sce_status sce_server_poll(sce_server s, uint64_t *ids, int32_t max, int32_t *n_done)
{
    if (!s || !n_done || max < 0 || (max > 0 && !ids)) return sfail(s, SCE_EINVAL, "bad argument");
    int32_t k = 0;
    while (k < max && !s->unpolled.empty()) {
        ids[k++] = s->unpolled.front();
        s->unpolled.pop_front();
    }
    *n_done = k;
    return SCE_OK;
}

sce_status sce_server_result(sce_server s, uint64_t id, double *x, double *v, double *F,
                             sce_diag *first, sce_diag *last)
{
    if (!s) return SCE_EINVAL;
    auto it = s->done.find(id);
    if (it == s->done.end()) return sfail(s, SCE_EINVAL, "request not finished or already fetched");
    const Result &r = it->second;
    if (x) std::memcpy(x, r.x.data(), r.x.size() * sizeof(double));
    if (v) std::memcpy(v, r.v.data(), r.v.size() * sizeof(double));
    if (F) std::memcpy(F, r.F.data(), r.F.size() * sizeof(double));
    if (first) fill_diag(first, r.diag, r.self_w, 0, r.dt, r.dim);
    if (last) fill_diag(last, r.diag + 8, r.self_w, r.n_steps, r.dt, r.dim);
    s->done.erase(it);
    return SCE_OK;
}

sce_status sce_server_stats(sce_server s, sce_server_report *o)
{
    if (!s || !o) return SCE_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->ticks = s->ticks;
    o->request_steps = s->request_steps;
    o->requests_done = s->requests_done;
    o->active = (int64_t)s->active.size();
    o->queued = (int64_t)s->queue.size();
    o->busy_s = s->busy;
    o->pairs = s->pairs;
    o->p50_step_s = weighted_pct(s->tick_lat, 0.50);
    o->p99_step_s = weighted_pct(s->tick_lat, 0.99);
    for (auto &e : s->tick_lat) o->max_step_s = std::max(o->max_step_s, e.first);
    o->gpu_p50_step_s = weighted_pct(s->tick_gpu, 0.50);
    o->gpu_p99_step_s = weighted_pct(s->tick_gpu, 0.99);
    std::vector<std::pair<double, int>> w;
    for (double x : s->waits) w.emplace_back(x, 1);
    o->p50_wait_s = weighted_pct(w, 0.50);
    o->p99_wait_s = weighted_pct(w, 0.99);
    o->hbm_used_bytes = (double)s->alloc.used;
    o->hbm_peak_bytes = (double)s->alloc.peak;
    return SCE_OK;
}

const char *sce_server_last_error(sce_server s) { return s ? s->err.c_str() : "null server"; }

void sce_server_destroy(sce_server s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    drop_graph(s);
    if (s->ev_a) (void)hipEventDestroy(s->ev_a);
    if (s->ev_b) (void)hipEventDestroy(s->ev_b);
    s->desc.release();
    s->dep.release();
    s->red.release();
    s->frc.release();
    s->slots.release();
    s->counts.release();
    s->stage.release();
    if (s->arena) (void)hipFree(s->arena);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
