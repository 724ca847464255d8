// Request server: continuous batching of assemblies and actions on resident
// models (C ABI in include/fem.h, "Request server").
//
// A model is a mesh with its form (Helmholtz, P_k, with the P1 fields kappa
// and f) made resident once: its sparsity and its Mat and Dat plans live in
// device memory for the server's lifetime (the paper keeps data on the
// device between parallel loops and pays setup once; its fixed per-call
// overheads are what batching amortises, "Experiments").
//
// Requests (an assembly: CSR matrix + right-hand side; or an action y = A x)
// queue in arrival order.  Whenever a slot is free, fem_server_poll takes a
// batch of queued requests (the queue head first, or, when asked, the
// requests of least estimated work, with a bound on how long the head can be
// passed over) as long as their outputs fit the budget, and queues the
// batch's work on the slot's stream as one persistent launch per kernel
// (Mat, source vector, action) and (dimension, degree): the workgroups of a
// launch take (request, row blocks) work items from a device counter, so
// small requests share one launch and large ones spread over the whole GPU.
// Batches admitted while others run overlap with them on the device.  The
// poll also retires batches whose completion event has fired.  Every block
// is computed by the same code, in the same order, as by the single-request
// kernels, and reads only its own request's data, so a result is bitwise the
// same alone and in any mix.
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <iterator>
#include <map>
#include <new>
#include <vector>

#include "fem_internal.h"

namespace {

fem_status sfail(fem_ctx *ctx, fem_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}
fem_status shed(fem_ctx *ctx, hipError_t e, const char *what)
{
    return sfail(ctx, e == hipErrorOutOfMemory ? FEM_E_NOMEM : FEM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}
#define SHIP(call, what)                                  \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return shed(ctx, e_, what); \
    } while (0)

// A resident model: deep copies of the caller's Set/Map/Dat descriptors (the
// device arrays they point to stay caller-owned), its sparsity and plans.
struct Model {
    fem_form form{}, src{};
    fem_set cells{}, verts{}, nodes{};
    fem_map cv{}, cn{};
    fem_dat X{}, kappa{}, f{};
    fem_args args{}, args_f{};
    fem_sparsity sp{};
    fem_plan *mplan = nullptr, *vplan = nullptr;
    int64_t resident = 0;
    int64_t nnz = 0, nrows = 0, ncells = 0;
};

struct Request {
    int32_t model = 0;
    int op = 0;
    const double *x = nullptr;
    double t_arrival = 0, t_admit = -1, t_done = -1;
    int state = 0;        // 0 queued, 1 running, 2 done, 3 released
    int slot = -1;
    double *values = nullptr, *vec = nullptr;
    int64_t bytes = 0;
    double work = 0;      // estimated work, for shortest-first admission
    int64_t off_values = -1, off_vec = -1;
};

// Device output arena: one allocation of the budget left after the resident
// models, carved first-fit into 256-byte aligned ranges on the host.  Taking
// and returning a range costs no driver call; a range is handed out again
// only after its request was released, i.e. after its kernels finished and
// the caller read the results.
struct Arena {
    char *base = nullptr;
    int64_t size = 0;
    std::map<int64_t, int64_t> free_;   // offset -> length, coalesced
    static int64_t round(int64_t b) { return (b + 255) / 256 * 256; }
    bool take(int64_t bytes, int64_t *off)
    {
        bytes = round(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const int64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        return false;
    }
    void give(int64_t off, int64_t bytes)
    {
        bytes = round(bytes ? bytes : 1);
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

}  // namespace

// Requests of one batch (at most FEM_SERVE_MAX_BATCH), and the descriptor
// memory of its launches: one (op, dimension, degree) group per launch.
constexpr int FEM_SERVE_MAX_BATCH = 64;
constexpr int FEM_SERVE_GROUPS = 18;     // 3 kernels x 6 (dimension, degree)

struct fem_server {
    fem_ctx *ctx = nullptr;
    hipStream_t home = nullptr;          // the context's stream at creation
    int64_t budget = 0, in_use = 0, resident = 0;
    int active = 0;                       // slots admission may use (<= streams.size())
    int share_cus = 1;                    // halve the Mat launch's grid while others run
    int max_batch = FEM_SERVE_MAX_BATCH;  // requests per batch
    double max_work = 1e8;                // estimated work per batch (a larger request runs alone)
    int order = FEM_SERVE_FIFO;           // which queued request admission takes next
    double max_wait = 0;                  // FEM_SERVE_SHORTEST: a head waiting this long goes first
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<std::vector<int64_t>> slot_reqs;   // the batch running on each slot (empty if free)
    std::vector<void *> ddesc, hdesc;    // per slot: launch descriptors (device, pinned host staging)
    size_t desc_bytes = 0;
    std::vector<Model *> models;
    std::vector<Request> reqs;
    std::deque<int64_t> queue;
    std::deque<int64_t> finished;         // completed, not yet handed out by take_completed
    Arena arena;                          // allocated at the first admission
};

// Work of a request, to order admission: cell visits of its plan times the
// local tensor size, plus the Mat values an assembly writes.
static double req_work(const Model &m, int op)
{
    const fem_plan &p = op == FEM_REQ_ASSEMBLE ? *m.mplan : *m.vplan;
    const double nl = p.nloc;
    return (double)p.cell_visits * nl * nl + (op == FEM_REQ_ASSEMBLE ? (double)m.nnz : 0.0);
}

// Arena bytes of a request's outputs, each range rounded as the arena carves it.
static int64_t req_bytes(const Model &m, int op)
{
    return Arena::round(8 * m.nrows ? 8 * m.nrows : 1) +
           (op == FEM_REQ_ASSEMBLE ? Arena::round(8 * m.nnz ? 8 * m.nnz : 1) : 0);
}

extern "C" {

static fem_status fem_server_create_impl(fem_ctx *ctx, int32_t slots, int64_t hbm_budget, fem_server **out);

fem_status fem_server_create(fem_ctx *ctx, int32_t slots, int64_t hbm_budget, fem_server **out)
{
    try {
        return fem_server_create_impl(ctx, slots, hbm_budget, out);
    } catch (...) {
        return femk::caught_status(ctx, "server_create");
    }
}

static fem_status fem_server_create_impl(fem_ctx *ctx, int32_t slots, int64_t hbm_budget, fem_server **out)
{
    if (!ctx) return FEM_E_ARG;
    if (!out || slots < 1 || slots > 64 || hbm_budget <= 0)
        return sfail(ctx, FEM_E_ARG, "server_create: slots must be 1..64 and the budget positive");
    fem_server *s = new (std::nothrow) fem_server;
    if (!s) return sfail(ctx, FEM_E_NOMEM, "server_create: host allocation");
    s->ctx = ctx;
    s->home = ctx->stream;
    s->budget = hbm_budget;
    s->active = slots;
    s->desc_bytes = FEM_SERVE_GROUPS * femk::batch_desc_bytes(FEM_SERVE_MAX_BATCH);
    for (int i = 0; i < slots; ++i) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        void *dd = nullptr, *hd = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = femk::mem_alloc(ctx->mem, ctx->stream, false, s->desc_bytes, &dd);
        if (e == hipSuccess) e = hipHostMalloc(&hd, s->desc_bytes, hipHostMallocDefault);
        if (st) s->streams.push_back(st);
        if (ev) s->events.push_back(ev);
        if (dd) s->ddesc.push_back(dd);
        if (hd) s->hdesc.push_back(hd);
        if (e != hipSuccess) {
            fem_server_destroy(s);
            return shed(ctx, e, "server_create: slot");
        }
        s->slot_reqs.emplace_back();
    }
    *out = s;
    return FEM_OK;
}

void fem_server_destroy(fem_server *s)
{
    if (!s) return;
    for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
    if (s->arena.base) femk::mem_free(s->ctx->mem, nullptr, false, s->arena.base);
    for (Model *m : s->models) {
        fem_plan_destroy(m->mplan);
        fem_plan_destroy(m->vplan);
        femk::mem_free(s->ctx->mem, nullptr, false, m->sp.row_ptr);
        femk::mem_free(s->ctx->mem, nullptr, false, m->sp.col_idx);
        delete m;
    }
    for (void *d : s->ddesc) femk::mem_free(s->ctx->mem, nullptr, false, d);
    for (void *h : s->hdesc) (void)hipHostFree(h);
    for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->ctx) s->ctx->stream = s->home;
    delete s;
}

static fem_status fem_server_add_model_impl(fem_server *s, const fem_form *form, const fem_args *args, int32_t *model_id,
                                int64_t *resident_bytes);

fem_status fem_server_add_model(fem_server *s, const fem_form *form, const fem_args *args, int32_t *model_id,
                                int64_t *resident_bytes)
{
    try {
        return fem_server_add_model_impl(s, form, args, model_id, resident_bytes);
    } catch (...) {
        return femk::caught_status(s ? s->ctx : nullptr, "server_add_model");
    }
}

static fem_status fem_server_add_model_impl(fem_server *s, const fem_form *form, const fem_args *args, int32_t *model_id,
                                int64_t *resident_bytes)
{
    if (!s) return FEM_E_ARG;
    fem_ctx *ctx = s->ctx;
    if (!form || !args || !model_id) return sfail(ctx, FEM_E_ARG, "add_model: NULL argument");
    if (s->arena.base) return sfail(ctx, FEM_E_ARG, "add_model: models must be added before the first admission");
    if (form->kind != FEM_HELMHOLTZ || form->prec != FEM_FP64 || form->dim != 1)
        return sfail(ctx, FEM_E_UNSUPPORTED, "add_model: the server runs the FP64 Helmholtz form");
    if (args->ncoeff < 2 || !args->coeff[0] || !args->coeff[1] || !args->cells || !args->cell_vertex ||
        !args->cell_node || !args->coords)
        return sfail(ctx, FEM_E_ARG, "add_model: args need cells, Maps, coords, coeff[0] = kappa, coeff[1] = f");
    Model *m = new (std::nothrow) Model;
    if (!m) return sfail(ctx, FEM_E_NOMEM, "add_model: host allocation");
    m->form = *form;
    m->src = *form;
    m->src.kind = FEM_SOURCE;
    m->cells = *args->cells;
    m->verts = *args->cell_vertex->to;
    m->nodes = *args->cell_node->to;
    m->cv = *args->cell_vertex;
    m->cv.from = &m->cells; m->cv.to = &m->verts;
    m->cn = *args->cell_node;
    m->cn.from = &m->cells; m->cn.to = &m->nodes;
    m->X = *args->coords; m->X.set = &m->verts;
    m->kappa = *args->coeff[0]; m->kappa.set = &m->verts;
    m->f = *args->coeff[1]; m->f.set = &m->verts;
    m->args.cells = &m->cells; m->args.cell_vertex = &m->cv; m->args.coords = &m->X; m->args.cell_node = &m->cn;
    m->args.coeff[0] = &m->kappa; m->args.ncoeff = 1;
    m->args_f = m->args;
    m->args_f.coeff[0] = &m->f;
    m->ncells = m->cells.size;
    m->nrows = m->nodes.size;
    ctx->stream = s->home;
    auto bail = [&](fem_status st) {
        fem_plan_destroy(m->mplan);
        fem_plan_destroy(m->vplan);
        femk::mem_free(ctx->mem, nullptr, false, m->sp.row_ptr);
        femk::mem_free(ctx->mem, nullptr, false, m->sp.col_idx);
        delete m;
        return st;
    };
    hipError_t e = femk::mem_alloc(ctx->mem, ctx->stream, false, sizeof(int64_t) * (m->nrows + 1),
                                   (void **)&m->sp.row_ptr);
    if (e != hipSuccess) return bail(shed(ctx, e, "add_model: alloc"));
    fem_status st = fem_build_sparsity(ctx, &m->cn, &m->cn, &m->sp, nullptr, nullptr);
    if (st != FEM_OK) return bail(st);
    e = femk::mem_alloc(ctx->mem, ctx->stream, false, sizeof(int32_t) * (m->sp.nnz ? m->sp.nnz : 1),
                        (void **)&m->sp.col_idx);
    if (e != hipSuccess) return bail(shed(ctx, e, "add_model: alloc"));
    if ((st = fem_build_sparsity(ctx, &m->cn, &m->cn, &m->sp, nullptr, nullptr)) != FEM_OK) return bail(st);
    if ((st = fem_plan_create(ctx, &m->form, &m->args, &m->sp, &m->mplan)) != FEM_OK) return bail(st);
    if ((st = fem_plan_create(ctx, &m->form, &m->args, nullptr, &m->vplan)) != FEM_OK) return bail(st);
    m->nnz = m->sp.nnz;
    m->resident = 12 * m->nnz + 8 * (m->nrows + 1) + (int64_t)m->mplan->bytes + (int64_t)m->vplan->bytes;
    if (s->resident + m->resident > s->budget)
        return bail(sfail(ctx, FEM_E_NOMEM, "add_model: resident data exceeds the HBM budget"));
    s->resident += m->resident;
    *model_id = (int32_t)s->models.size();
    s->models.push_back(m);
    if (resident_bytes) *resident_bytes = m->resident;
    return FEM_OK;
}

static fem_status fem_server_submit_impl(fem_server *s, int32_t model, int32_t op, const double *x, double arrival_time,
                             int64_t *req_id);

fem_status fem_server_submit(fem_server *s, int32_t model, int32_t op, const double *x, double arrival_time,
                             int64_t *req_id)
{
    try {
        return fem_server_submit_impl(s, model, op, x, arrival_time, req_id);
    } catch (...) {
        return femk::caught_status(s ? s->ctx : nullptr, "server_submit");
    }
}

static fem_status fem_server_submit_impl(fem_server *s, int32_t model, int32_t op, const double *x, double arrival_time,
                             int64_t *req_id)
{
    if (!s) return FEM_E_ARG;
    fem_ctx *ctx = s->ctx;
    if (model < 0 || model >= (int32_t)s->models.size()) return sfail(ctx, FEM_E_ARG, "submit: unknown model");
    if (op != FEM_REQ_ASSEMBLE && op != FEM_REQ_ACTION) return sfail(ctx, FEM_E_ARG, "submit: unknown operation");
    if (op == FEM_REQ_ACTION && !x && s->models[model]->nrows > 0) return sfail(ctx, FEM_E_ARG, "submit: action needs x");
    const int64_t bytes = req_bytes(*s->models[model], op);
    if (bytes > (s->budget - s->resident) / 256 * 256)   // the output arena's size
        return sfail(ctx, FEM_E_NOMEM, "submit: the request's outputs can never fit the HBM budget");
    Request r;
    r.model = model; r.op = op; r.x = x; r.t_arrival = arrival_time; r.bytes = bytes;
    r.work = req_work(*s->models[model], op);
    s->reqs.push_back(r);
    s->queue.push_back((int64_t)s->reqs.size() - 1);
    if (req_id) *req_id = (int64_t)s->reqs.size() - 1;
    return FEM_OK;
}

// Queues one batch's work on a slot: per (kernel, dimension, degree), one
// launch over every request of the batch that needs it.
static fem_status launch_batch_on(fem_server *s, int slot, const std::vector<int64_t> &batch, bool busy)
{
    fem_ctx *ctx = s->ctx;
    hipStream_t st = s->streams[slot];
    // group: kernel (op), dimension and degree
    std::map<int, std::vector<femk::AsmArgs>> groups;
    for (int64_t rid : batch) {
        const Request &r = s->reqs[rid];
        const Model &m = *s->models[r.model];
        femk::AsmArgs a{};
        a.cell_vertex = m.cv.values;
        a.coords = m.X.data;
        a.cell_node = m.cn.values;
        a.cstiff = 1.0;   // the Helmholtz form
        a.cmass = 1.0;
        a.num_cus = ctx->num_cus;
        const int dk = ((int)m.form.cell - 2) * 3 + (m.form.degree - 1);
        if (r.op == FEM_REQ_ASSEMBLE) {
            femk::AsmArgs am = a;
            am.plan = m.mplan; am.coeff = m.kappa.data; am.row_ptr = m.sp.row_ptr; am.out = r.values;
            groups[0 * 6 + dk].push_back(am);
            femk::AsmArgs av = a;
            av.plan = m.vplan; av.coeff = m.f.data; av.out = r.vec;
            groups[1 * 6 + dk].push_back(av);
        } else {
            femk::AsmArgs aa = a;
            aa.plan = m.vplan; aa.coeff = m.kappa.data; aa.x = r.x; aa.out = r.vec;
            groups[2 * 6 + dk].push_back(aa);
        }
    }
    // the Mat launch fills every CU while its work lasts; while other batches
    // run or requests wait it takes half of them
    const int cus = ctx->num_cus;
    const int mat_grid = busy && s->share_cus ? (cus > 1 ? cus / 2 : 1) : cus;
    size_t off = 0;
    for (auto &kv : groups) {
        const int op = kv.first / 6;
        const std::vector<femk::AsmArgs> &gr = kv.second;
        char *h = static_cast<char *>(s->hdesc[slot]) + off, *d = static_cast<char *>(s->ddesc[slot]) + off;
        SHIP(femk::launch_batch(op, gr.data(), (int)gr.size(), op == 0 ? mat_grid : cus, h, d, st),
             "poll: batched launch");
        off += femk::batch_desc_bytes((int)gr.size());
    }
    SHIP(hipEventRecord(s->events[slot], st), "poll: event");
    return FEM_OK;
}

static fem_status fem_server_poll_impl(fem_server *s, double now, int32_t *completed, int32_t *running, int32_t *queued);

fem_status fem_server_poll(fem_server *s, double now, int32_t *completed, int32_t *running, int32_t *queued)
{
    try {
        return fem_server_poll_impl(s, now, completed, running, queued);
    } catch (...) {
        return femk::caught_status(s ? s->ctx : nullptr, "server_poll");
    }
}

static fem_status fem_server_poll_impl(fem_server *s, double now, int32_t *completed, int32_t *running, int32_t *queued)
{
    if (!s) return FEM_E_ARG;
    fem_ctx *ctx = s->ctx;
    int32_t done = 0;
    // retire finished batches
    for (size_t k = 0; k < s->streams.size(); ++k) {
        if (s->slot_reqs[k].empty()) continue;
        const hipError_t e = hipEventQuery(s->events[k]);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return shed(ctx, e, "poll: request failed on the device");
        for (int64_t q : s->slot_reqs[k]) {
            Request &r = s->reqs[q];
            r.state = 2;
            r.t_done = now;
            s->finished.push_back(q);
            ++done;
        }
        s->slot_reqs[k].clear();
    }
    // the output arena: everything the resident models leave of the budget
    if (!s->arena.base && !s->queue.empty()) {
        const int64_t size = (s->budget - s->resident) / 256 * 256;
        SHIP(femk::mem_alloc(ctx->mem, ctx->stream, false, size, (void **)&s->arena.base), "poll: output arena");
        s->arena.size = size;
        s->arena.free_[0] = size;
    }
    // admit batches while a slot is free: the next request is the queue head
    // (FIFO), or the queued request of least estimated work (ties: the
    // earlier) unless the head has waited max_wait or longer; a batch closes
    // at max_batch requests or at the first request whose outputs do not fit
    while (!s->queue.empty()) {
        int slot = -1;
        for (int k = 0; k < s->active; ++k)
            if (s->slot_reqs[k].empty()) { slot = k; break; }
        if (slot < 0) break;
        std::vector<int64_t> batch;
        double batch_work = 0.0;
        while (!s->queue.empty() && (int)batch.size() < s->max_batch) {
            auto pick = s->queue.begin();
            if (s->order == FEM_SERVE_SHORTEST && now - s->reqs[*pick].t_arrival < s->max_wait)
                for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
                    if (s->reqs[*it].work < s->reqs[*pick].work) pick = it;
            const int64_t rid = *pick;
            Request &r = s->reqs[rid];
            if (!batch.empty() && batch_work + r.work > s->max_work) break;
            if (s->resident + s->in_use + r.bytes > s->budget) break;
            const Model &m = *s->models[r.model];
            // outputs from the arena (fragmentation may refuse what the
            // budget allows: then wait for releases)
            int64_t ov = -1, ob = -1;
            if (!s->arena.take(8 * m.nrows, &ob)) break;
            if (r.op == FEM_REQ_ASSEMBLE && !s->arena.take(8 * m.nnz, &ov)) {
                s->arena.give(ob, 8 * m.nrows);
                break;
            }
            r.off_vec = ob; r.off_values = ov;
            r.vec = reinterpret_cast<double *>(s->arena.base + ob);
            r.values = ov >= 0 ? reinterpret_cast<double *>(s->arena.base + ov) : nullptr;
            r.state = 1;
            r.slot = slot;
            r.t_admit = now;
            s->in_use += r.bytes;
            s->queue.erase(pick);
            batch.push_back(rid);
            batch_work += r.work;
        }
        if (batch.empty()) break;
        bool busy = !s->queue.empty();
        for (const auto &b : s->slot_reqs) busy |= !b.empty();
        fem_status fs = launch_batch_on(s, slot, batch, busy);
        s->slot_reqs[slot] = batch;
        if (fs != FEM_OK) return fs;
    }
    int32_t run = 0;
    for (const auto &b : s->slot_reqs) run += (int32_t)b.size();
    if (completed) *completed = done;
    if (running) *running = run;
    if (queued) *queued = (int32_t)s->queue.size();
    return FEM_OK;
}

fem_status fem_server_result(fem_server *s, int64_t req, const double **values, const double **vec, double *t_admit,
                             double *t_done)
{
    if (!s) return FEM_E_ARG;
    if (req < 0 || req >= (int64_t)s->reqs.size()) return sfail(s->ctx, FEM_E_ARG, "result: unknown request");
    const Request &r = s->reqs[req];
    if (r.state != 2) return sfail(s->ctx, FEM_E_ARG, "result: request %lld is not complete", (long long)req);
    if (values) *values = r.values;
    if (vec) *vec = r.vec;
    if (t_admit) *t_admit = r.t_admit;
    if (t_done) *t_done = r.t_done;
    return FEM_OK;
}

fem_status fem_server_release(fem_server *s, int64_t req)
{
    if (!s) return FEM_E_ARG;
    fem_ctx *ctx = s->ctx;
    if (req < 0 || req >= (int64_t)s->reqs.size()) return sfail(ctx, FEM_E_ARG, "release: unknown request");
    Request &r = s->reqs[req];
    if (r.state != 2) return sfail(ctx, FEM_E_ARG, "release: request %lld is not complete", (long long)req);
    const Model &m = *s->models[r.model];
    if (r.off_values >= 0) s->arena.give(r.off_values, 8 * m.nnz);
    if (r.off_vec >= 0) s->arena.give(r.off_vec, 8 * m.nrows);
    r.values = r.vec = nullptr;
    r.off_values = r.off_vec = -1;
    s->in_use -= r.bytes;
    r.state = 3;
    return FEM_OK;
}

fem_status fem_server_take_completed(fem_server *s, int64_t *ids, int32_t cap, int32_t *n)
{
    if (!s || !n || (cap > 0 && !ids)) return FEM_E_ARG;
    int32_t k = 0;
    while (k < cap && !s->finished.empty()) {
        ids[k++] = s->finished.front();
        s->finished.pop_front();
    }
    *n = k;
    return FEM_OK;
}

fem_status fem_server_configure(fem_server *s, int32_t slots, int32_t share_cus)
{
    if (!s) return FEM_E_ARG;
    if (slots < 1 || slots > (int32_t)s->streams.size())
        return sfail(s->ctx, FEM_E_ARG, "configure: slots must be 1..%d", (int)s->streams.size());
    s->active = slots;   // running requests on higher slots finish normally
    s->share_cus = share_cus != 0;
    return FEM_OK;
}

fem_status fem_server_set_batch(fem_server *s, int32_t max_requests, double max_work)
{
    if (!s) return FEM_E_ARG;
    if (max_requests < 1 || max_requests > FEM_SERVE_MAX_BATCH)
        return sfail(s->ctx, FEM_E_ARG, "set_batch: 1..%d requests per batch", FEM_SERVE_MAX_BATCH);
    if (!(max_work > 0)) return sfail(s->ctx, FEM_E_ARG, "set_batch: max_work must be positive");
    s->max_batch = max_requests;
    s->max_work = max_work;
    return FEM_OK;
}

fem_status fem_server_set_order(fem_server *s, int32_t order, double max_wait)
{
    if (!s) return FEM_E_ARG;
    if (order != FEM_SERVE_FIFO && order != FEM_SERVE_SHORTEST)
        return sfail(s->ctx, FEM_E_ARG, "set_order: unknown order");
    if (!(max_wait >= 0)) return sfail(s->ctx, FEM_E_ARG, "set_order: max_wait must be >= 0");
    s->order = order;
    s->max_wait = max_wait;
    return FEM_OK;
}

fem_status fem_server_model_info(const fem_server *s, int32_t model, int64_t *cells, int64_t *nrows, int64_t *nnz,
                                 const int64_t **row_ptr, const int32_t **col_idx)
{
    if (!s || model < 0 || model >= (int32_t)s->models.size()) return FEM_E_ARG;
    const Model &m = *s->models[model];
    if (cells) *cells = m.ncells;
    if (nrows) *nrows = m.nrows;
    if (nnz) *nnz = m.nnz;
    if (row_ptr) *row_ptr = m.sp.row_ptr;
    if (col_idx) *col_idx = m.sp.col_idx;
    return FEM_OK;
}

}  // extern "C"
