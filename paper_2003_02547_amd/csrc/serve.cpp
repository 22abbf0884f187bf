// Continuous-batching request server over the batched IPM kernels.
//
// A request is one OCP QP (Section 2.2) packed once by the client into a
// relocatable blob (oqp_pack).  The server admits a request when a block of
// the caller's device buffer large enough for its data, iterate and
// workspace records is free (first-fit, coalescing on release), so admission
// is by HBM footprint.  oqp_server_progress retires finished launches (one
// event per launch) and, on every idle stream, launches the queued requests
// of one kernel group together: a request that arrives while the device is
// busy joins the next launch, launches run concurrently on the caller's
// streams, and their size follows the load.
// The IPM state of a request stays in its device block from admission to
// release; every IPM iteration runs inside one kernel launch.
//
// Memory: every structure lives in caller memory (host memory must be
// page-locked so the per-launch descriptor and status copies are
// asynchronous).  The only driver objects created are one HIP event per
// launch slot, destroyed by oqp_server_destroy.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstring>

#include "../../include/oqp.h"
#include "arena.h"
#include "internal.h"
#include "layout.h"

using oqp::DevStat;
using oqp::InstDesc;
using oqp::Layout;

namespace {

constexpr uint32_t kPackMagic = 0x4f515031u;  // "OQP1"

// Header of a packed request; offsets in bytes from the blob start.
struct PackHdr {
    uint32_t magic;
    int32_t variant;  // kernel group
    int32_t N;
    int32_t nc;
    int32_t nx, nu, ng, soft;  // padded stage sizes of the records; soft layout
    int64_t data_doubles, iter_doubles, work_doubles;
    int64_t dims_off, slots_off, data_off;
    int64_t total;
    int64_t soft_off;  // soft layout: ns per stage, then the device slot of each slack
    int32_t nsoft, pad;
};

size_t dev_footprint(const PackHdr* h)
{
    return align_up(sizeof(double) * h->data_doubles, 256) + align_up(sizeof(double) * h->iter_doubles, 256) +
           align_up(sizeof(double) * h->work_doubles, 256);
}

int read_hdr(const void* packed, const PackHdr** out)
{
    if (!packed) return fail(OQP_EINVAL, "packed request is NULL");
    if ((uintptr_t)packed % 8) return fail(OQP_EINVAL, "packed request not 8-byte aligned");
    const PackHdr* h = (const PackHdr*)packed;
    if (h->magic != kPackMagic) return fail(OQP_EINVAL, "not a packed request (bad magic)");
    // kernel groups: one per kernel choice, and again for the soft builds
    if (h->variant < 0 || h->variant >= 2 * group_count()) return fail(OQP_EINVAL, "packed request: bad kernel group");
    *out = h;
    return OQP_OK;
}

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum { RQ_FREE = 0, RQ_QUEUED, RQ_RUNNING, RQ_DONE };

struct Request {
    int state;
    uint32_t gen;
    const PackHdr* hdr;
    size_t dev_off;    // bytes from the arena start
    size_t dev_bytes;
    int group;         // launch slot while running
    int gpos;          // position inside that launch
    int next;          // FIFO link while queued, free-list link while free
    int64_t tag;       // caller's index (replay)
    int64_t t_submit, t_done;
    DevStat stat;
    int resume;        // iteration blocks: the request continues from its iterate records
    int iters_done;    // iteration blocks: iterations and refinement corrections so far
    int ir_done;
};

struct Group {
    int busy;
    int stream;
    int count;
    int next;              // per-stream FIFO link
    hipEvent_t ev;
    InstDesc* hdesc;       // page-locked host
    DevStat* hstat;        // page-locked host
    InstDesc* ddesc;       // device
    DevStat* dstat;        // device
    int* req;              // request slot of each launched instance
};

}  // namespace

struct oqp_server {
    oqp_server_cfg cfg;
    oqp_arg arg;
    int nvar;
    int nstreams;
    hipStream_t streams[OQP_SERVER_MAX_STREAMS];
    int sq_head[OQP_SERVER_MAX_STREAMS], sq_tail[OQP_SERVER_MAX_STREAMS], sq_len[OQP_SERVER_MAX_STREAMS];
    Request* req;
    int free_head;          // stack of free request slots (linked by next)
    int q_head, q_tail;     // FIFO of queued requests
    Arena mem;              // free device ranges of the arena
    Group* grp;
    int* done_ring;         // requests completed by progress, drained by replay
    int done_head, done_len;
    char* arena;
    size_t arena_bytes;
    double* staging;
    uint64_t submitted, rejected, completed, launches;
    int queued, running, done;
};

namespace {

struct SrvPlan {
    size_t host, h_req, h_fr, h_grp, h_gdesc, h_gstat, h_greq, h_ring, h_stage;
    size_t dev_fixed, d_desc, d_stat;
};

int check_cfg(const oqp_server_cfg* c)
{
    if (!c) return fail(OQP_EINVAL, "server cfg is NULL");
    if (c->max_requests < 1 || c->max_launch < 1 || c->max_groups < 1)
        return fail(OQP_EINVAL, "server cfg: max_requests, max_launch and max_groups must be >= 1");
    if (c->max_requests > (1 << 20) || c->max_launch > 65536 || c->max_groups > 4096)
        return fail(OQP_EINVAL, "server cfg: sizes too large");
    if (c->iter_block < 0) return fail(OQP_EINVAL, "server cfg: iter_block must be >= 0");
    return OQP_OK;
}

SrvPlan srv_plan(const oqp_server_cfg* c)
{
    SrvPlan p{};
    size_t h = align_up(sizeof(oqp_server), 64);
    p.h_req = h; h = align_up(h + sizeof(Request) * c->max_requests, 64);
    p.h_fr = h; h = align_up(h + sizeof(ArenaRange) * (c->max_requests + 2), 64);
    p.h_grp = h; h = align_up(h + sizeof(Group) * c->max_groups, 64);
    p.h_gdesc = h; h = align_up(h + sizeof(InstDesc) * c->max_launch * (size_t)c->max_groups, 64);
    p.h_gstat = h; h = align_up(h + sizeof(DevStat) * c->max_launch * (size_t)c->max_groups, 64);
    p.h_greq = h; h = align_up(h + sizeof(int) * c->max_launch * (size_t)c->max_groups, 64);
    p.h_ring = h; h = align_up(h + sizeof(int) * c->max_requests, 64);
    p.h_stage = h; h = align_up(h + c->staging_bytes, 64);
    p.host = h;
    size_t g = 0;
    p.d_desc = g; g = align_up(g + sizeof(InstDesc) * c->max_launch * (size_t)c->max_groups, 256);
    p.d_stat = g; g = align_up(g + sizeof(DevStat) * c->max_launch * (size_t)c->max_groups, 256);
    p.dev_fixed = g;
    return p;
}

int ticket_slot(const oqp_server* s, uint64_t ticket)
{
    const int slot = (int)(ticket & 0xffffffffu);
    const uint32_t gen = (uint32_t)(ticket >> 32);
    if (slot < 0 || slot >= s->cfg.max_requests) return -1;
    const Request& r = s->req[slot];
    if (r.state == RQ_FREE || r.gen != gen) return -1;
    return slot;
}

// Retire every finished launch (oldest first on each stream).
int retire(oqp_server* s, int* ncompleted)
{
    for (int k = 0; k < s->nstreams; ++k) {
        while (s->sq_len[k] > 0) {
            const int gi = s->sq_head[k];
            Group& g = s->grp[gi];
            hipError_t e = hipEventQuery(g.ev);
            if (e == hipErrorNotReady) {
                (void)hipGetLastError();  // not an error: clear it for later callers
                break;
            }
            if (e != hipSuccess) return fail(OQP_EDEVICE, "server: hipEventQuery: %s", hipGetErrorString(e));
            const int64_t t = now_ns();
            int finished = 0;
            for (int j = 0; j < g.count; ++j) {
                const int slot = g.req[j];
                Request& r = s->req[slot];
                r.stat = g.hstat[j];
                r.iters_done += r.stat.iters;
                r.ir_done += r.stat.ir_steps;
                r.stat.iters = r.iters_done;
                r.stat.ir_steps = r.ir_done;
                if (s->cfg.iter_block > 0 && r.stat.status == oqp::ST_MAX_ITER && r.iters_done < s->arg.iter_max) {
                    // iteration block used up: queue again, ahead of the
                    // requests that have not started
                    r.state = RQ_QUEUED;
                    r.resume = 1;
                    r.next = s->q_head;
                    s->q_head = slot;
                    if (s->q_tail < 0) s->q_tail = slot;
                    ++s->queued;
                    continue;
                }
                r.state = RQ_DONE;
                r.t_done = t;
                s->done_ring[(s->done_head + s->done_len) % s->cfg.max_requests] = slot;
                ++s->done_len;
                ++finished;
            }
            s->running -= g.count;
            s->done += finished;
            s->completed += finished;
            if (ncompleted) *ncompleted += finished;
            g.busy = 0;
            s->sq_head[k] = g.next;
            --s->sq_len[k];
        }
    }
    return OQP_OK;
}

int free_group(const oqp_server* s)
{
    for (int i = 0; i < s->cfg.max_groups; ++i)
        if (!s->grp[i].busy) return i;
    return -1;
}

// An idle launch stream (none of its launches in flight), or -1.  Stream 0
// is kept for solution fetches.  A launch therefore never queues behind
// another one: while every stream is busy, arriving requests accumulate and
// the next idle stream takes all of them (of one kernel group) at once, so
// launches grow with the load.
int pick_stream(const oqp_server* s)
{
    for (int k = 1; k < s->nstreams; ++k)
        if (s->sq_len[k] == 0) return k;
    return -1;
}

// Launch one group: the queued requests of variant v, oldest first.
int launch_group(oqp_server* s, int v, int gi, int k)
{
    Group& g = s->grp[gi];
    hipStream_t st = s->streams[k];
    double* base = (double*)s->arena;
    int cnt = 0;
    int prev = -1, r = s->q_head;
    while (r >= 0 && cnt < s->cfg.max_launch) {
        Request& q = s->req[r];
        const int nxt = q.next;
        if (q.hdr->variant != v) {
            prev = r;
            r = nxt;
            continue;
        }
        // unlink from the queue
        if (prev < 0) s->q_head = nxt; else s->req[prev].next = nxt;
        if (s->q_tail == r) s->q_tail = prev;
        const PackHdr* h = q.hdr;
        const size_t db = align_up(sizeof(double) * h->data_doubles, 256);
        const size_t ib = align_up(sizeof(double) * h->iter_doubles, 256);
        InstDesc& d = g.hdesc[cnt];
        d.data = (int64_t)(q.dev_off / sizeof(double));
        d.iter = (int64_t)((q.dev_off + db) / sizeof(double));
        d.work = (int64_t)((q.dev_off + db + ib) / sizeof(double));
        d.N = h->N;
        d.nc = h->nc + h->nsoft;  // one-sided rows / 2: constraint rows and slack bounds
        d.index = cnt;
        d.resume = q.resume;
        d.nx = h->nx;
        d.nu = h->nu;
        d.ng = h->ng;
        // iteration blocks: at most iter_block iterations, within what is
        // left of the request's iteration limit
        d.itcap = s->cfg.iter_block > 0 ? std::min(s->cfg.iter_block, s->arg.iter_max - q.iters_done) : 0;
        d.nuN = h->nu;  // padded size: the server's kernels read the whole block
        d.pad = 0;
        if (!q.resume) {
            hipError_t e = hipMemcpyAsync(s->arena + q.dev_off, (const char*)h + h->data_off,
                                          sizeof(double) * h->data_doubles, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) return fail(OQP_EDEVICE, "server: request upload: %s", hipGetErrorString(e));
        }
        q.state = RQ_RUNNING;
        q.group = gi;
        q.gpos = cnt;
        g.req[cnt] = r;
        ++cnt;
        r = nxt;
    }
    if (cnt == 0) return OQP_OK;
    g.busy = 1;
    g.count = cnt;
    g.stream = k;
    g.next = -1;
    hipError_t e = hipMemcpyAsync(g.ddesc, g.hdesc, sizeof(InstDesc) * cnt, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "server: descriptor upload: %s", hipGetErrorString(e));
    // groups at and above group_count() hold requests with slacks
    const int kg = v % group_count();
    const int km = v >= group_count() ? oqp::KM_SOFT : kernel_build(s->arg.mode);
    oqp::KParams P = make_params(s->arg, oqp::KMODE_SOLVE, 0.0);
    if (group_launch(kg, km, g.ddesc, g.hdesc, cnt, base, base, base, base, g.dstat, P, st))
        return fail(OQP_EDEVICE, "server: kernel launch failed for group %d", v);
    if (km == oqp::KM_MIXED) {
        P.mode = oqp::KMODE_FALLBACK;
        P.ir_max = 0;  // the fallback is the plain FP64 path (no refinement)
        P.warm = 0;    // a handed-over iterate is resumed; any other starts cold
        if (group_launch(kg, oqp::KM_F64, g.ddesc, g.hdesc, cnt, base, base, base, base, g.dstat, P, st))
            return fail(OQP_EDEVICE, "server: fallback launch failed for group %d", v);
    }
    e = hipMemcpyAsync(g.hstat, g.dstat, sizeof(DevStat) * cnt, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(g.ev, st);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "server: status copy: %s", hipGetErrorString(e));
    if (s->sq_len[k] == 0) s->sq_head[k] = gi; else s->grp[s->sq_tail[k]].next = gi;
    s->sq_tail[k] = gi;
    ++s->sq_len[k];
    s->queued -= cnt;
    s->running += cnt;
    ++s->launches;
    return OQP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------

static void pack_sizes(const oqp_qp* q, const KSel& ks, PackHdr* h)
{
    const oqp_dims* d = q->dims;
    const bool soft = dims_soft(d);
    const Layout L = oqp::make_layout(ks.nx, ks.nu, ks.ng, soft);
    int nc = 0, ns = 0;
    for (int n = 0; n <= d->N; ++n) {
        nc += d->nbu[n] + d->nbx[n] + d->ng[n];
        ns += d->ns[n];
    }
    std::memset(h, 0, sizeof(*h));
    h->magic = kPackMagic;
    h->variant = ks.group + (soft ? group_count() : 0);
    h->soft = soft ? 1 : 0;
    h->nsoft = ns;
    h->N = d->N;
    h->nc = nc;
    h->nx = ks.nx;
    h->nu = ks.nu;
    h->ng = ks.ng;
    h->data_doubles = (int64_t)(d->N + 1) * L.SREC;
    h->iter_doubles = (int64_t)(d->N + 1) * L.IREC;
    h->work_doubles = (int64_t)(d->N + 1) * L.WREC;
    size_t o = align_up(sizeof(PackHdr), 64);
    h->dims_off = (int64_t)o;
    o = align_up(o + sizeof(int) * 5 * (d->N + 1), 64);
    h->slots_off = (int64_t)o;
    o = align_up(o + sizeof(int) * (nc + 1), 64);
    h->soft_off = (int64_t)o;
    o = align_up(o + sizeof(int) * (soft ? d->N + 1 + ns : 1), 64);
    h->data_off = (int64_t)o;
    o = align_up(o + sizeof(double) * h->data_doubles, 64);
    h->total = (int64_t)o;
}

extern "C" int oqp_pack_bytes(const oqp_qp* qp, size_t* bytes)
{
    if (!qp || !bytes) return fail(OQP_EINVAL, "oqp_pack_bytes: NULL argument");
    KSel ks;
    if (select_kernel(qp->dims, &ks)) return fail(OQP_EINVAL, "oqp_pack_bytes: no kernel covers the stage sizes");
    PackHdr h;
    pack_sizes(qp, ks, &h);
    *bytes = (size_t)h.total;
    return OQP_OK;
}

extern "C" int oqp_pack(const oqp_qp* qp, void* mem, size_t bytes)
{
    if (!qp || !mem) return fail(OQP_EINVAL, "oqp_pack: NULL argument");
    if ((uintptr_t)mem % 64) return fail(OQP_EINVAL, "oqp_pack: memory not 64-byte aligned");
    KSel ks;
    if (select_kernel(qp->dims, &ks)) return fail(OQP_EINVAL, "oqp_pack: no kernel covers the stage sizes");
    PackHdr h;
    pack_sizes(qp, ks, &h);
    if (bytes < (size_t)h.total) return fail(OQP_ENOMEM, "oqp_pack: %zu < %lld bytes", bytes, (long long)h.total);
    char* b = (char*)mem;
    std::memset(b, 0, (size_t)h.data_off);
    std::memcpy(b, &h, sizeof(h));
    const oqp_dims* d = qp->dims;
    int* dims5 = (int*)(b + h.dims_off);
    for (int n = 0; n <= d->N; ++n) {
        dims5[0 * (d->N + 1) + n] = d->nx[n];
        dims5[1 * (d->N + 1) + n] = d->nu[n];
        dims5[2 * (d->N + 1) + n] = d->nbu[n];
        dims5[3 * (d->N + 1) + n] = d->nbx[n];
        dims5[4 * (d->N + 1) + n] = d->ng[n];
    }
    int* soft = (int*)(b + h.soft_off);
    if (h.soft)
        for (int n = 0; n <= d->N; ++n) soft[n] = d->ns[n];
    return pack_records(qp, oqp::make_layout(h.nx, h.nu, h.ng, h.soft != 0), (double*)(b + h.data_off),
                        (int*)(b + h.slots_off), h.soft ? soft + d->N + 1 : nullptr);
}

extern "C" int oqp_pack_footprint(const void* packed, size_t* dev_bytes, int* variant)
{
    const PackHdr* h;
    int rc = read_hdr(packed, &h);
    if (rc) return rc;
    if (dev_bytes) *dev_bytes = dev_footprint(h);
    if (variant) *variant = h->variant;
    return OQP_OK;
}

// ---------------------------------------------------------------------------
// server
// ---------------------------------------------------------------------------

extern "C" void oqp_server_cfg_default(oqp_server_cfg* c)
{
    if (!c) return;
    c->max_requests = 1024;
    c->max_launch = 256;
    c->max_groups = 256;
    c->staging_bytes = (size_t)16 << 20;
    c->iter_block = 0;
}

extern "C" int oqp_server_bytes(const oqp_server_cfg* cfg, size_t* host_bytes, size_t* dev_fixed_bytes)
{
    int rc = check_cfg(cfg);
    if (rc) return rc;
    const SrvPlan p = srv_plan(cfg);
    if (host_bytes) *host_bytes = p.host;
    if (dev_fixed_bytes) *dev_fixed_bytes = p.dev_fixed;
    return OQP_OK;
}

extern "C" int oqp_server_init(const oqp_server_cfg* cfg, const oqp_arg* arg, void* host_mem, size_t host_bytes,
                               void* dev_mem, size_t dev_bytes, void* const* streams, int nstreams,
                               oqp_server** out)
{
    int rc = check_cfg(cfg);
    if (rc) return rc;
    rc = check_arg(arg);
    if (rc) return rc;
    if (arg->cond_N != 0 || arg->warm_start != 0 || arg->mode == OQP_MODE_ROBUST || arg->mode == OQP_MODE_BALANCE)
        return fail(OQP_EINVAL, "oqp_server_init: partial condensing, warm start, robust and balance modes are batch options");
    if (cfg->iter_block > 0 && arg->mode != OQP_MODE_F64)
        return fail(OQP_EINVAL, "oqp_server_init: iteration blocks need the FP64 mode");
    if (!host_mem || !dev_mem || !streams || !out) return fail(OQP_EINVAL, "oqp_server_init: NULL argument");
    if (nstreams < 2 || nstreams > OQP_SERVER_MAX_STREAMS)
        return fail(OQP_EINVAL, "oqp_server_init: need 2..%d streams", OQP_SERVER_MAX_STREAMS);
    if ((uintptr_t)host_mem % 64) return fail(OQP_EINVAL, "oqp_server_init: host memory not 64-byte aligned");
    if ((uintptr_t)dev_mem % 256) return fail(OQP_EINVAL, "oqp_server_init: device memory not 256-byte aligned");
    const SrvPlan p = srv_plan(cfg);
    if (host_bytes < p.host) return fail(OQP_ENOMEM, "oqp_server_init: host %zu < %zu", host_bytes, p.host);
    if (dev_bytes < p.dev_fixed + 256)
        return fail(OQP_ENOMEM, "oqp_server_init: device %zu leaves no arena (fixed part %zu)", dev_bytes, p.dev_fixed);
    hipPointerAttribute_t pa;
    hipError_t e = hipPointerGetAttributes(&pa, host_mem);
    if (e != hipSuccess || pa.type != hipMemoryTypeHost) {
        (void)hipGetLastError();
        return fail(OQP_EINVAL, "oqp_server_init: host memory must be page-locked (hipHostMalloc)");
    }
    char* h = (char*)host_mem;
    char* g = (char*)dev_mem;
    oqp_server* s = (oqp_server*)h;
    std::memset(s, 0, sizeof(*s));
    s->cfg = *cfg;
    s->arg = *arg;
    s->nvar = group_count();
    s->nstreams = nstreams;
    for (int k = 0; k < nstreams; ++k) s->streams[k] = (hipStream_t)streams[k];
    s->req = (Request*)(h + p.h_req);
    s->grp = (Group*)(h + p.h_grp);
    s->done_ring = (int*)(h + p.h_ring);
    s->staging = (double*)(h + p.h_stage);
    for (int i = 0; i < cfg->max_requests; ++i) {
        std::memset(&s->req[i], 0, sizeof(Request));
        s->req[i].next = i + 1 < cfg->max_requests ? i + 1 : -1;
    }
    s->free_head = 0;
    s->q_head = s->q_tail = -1;
    s->arena = g + p.dev_fixed;
    s->arena_bytes = (dev_bytes - p.dev_fixed) / 256 * 256;
    arena_reset(s->mem, (ArenaRange*)(h + p.h_fr), s->arena_bytes);
    InstDesc* hd = (InstDesc*)(h + p.h_gdesc);
    DevStat* hs = (DevStat*)(h + p.h_gstat);
    int* gr = (int*)(h + p.h_greq);
    InstDesc* dd = (InstDesc*)(g + p.d_desc);
    DevStat* ds = (DevStat*)(g + p.d_stat);
    for (int i = 0; i < cfg->max_groups; ++i) {
        Group& gp = s->grp[i];
        std::memset(&gp, 0, sizeof(gp));
        gp.hdesc = hd + (size_t)i * cfg->max_launch;
        gp.hstat = hs + (size_t)i * cfg->max_launch;
        gp.req = gr + (size_t)i * cfg->max_launch;
        gp.ddesc = dd + (size_t)i * cfg->max_launch;
        gp.dstat = ds + (size_t)i * cfg->max_launch;
        e = hipEventCreateWithFlags(&gp.ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(s->grp[j].ev);
            return fail(OQP_EDEVICE, "oqp_server_init: hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    *out = s;
    return OQP_OK;
}

extern "C" int oqp_server_destroy(oqp_server* s)
{
    if (!s) return fail(OQP_EINVAL, "oqp_server_destroy: NULL server");
    int rc = OQP_OK;
    for (int k = 0; k < s->nstreams; ++k) {
        hipError_t e = hipStreamSynchronize(s->streams[k]);
        if (e != hipSuccess && rc == OQP_OK) rc = fail(OQP_EDEVICE, "oqp_server_destroy: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < s->cfg.max_groups; ++i) (void)hipEventDestroy(s->grp[i].ev);
    s->nstreams = 0;
    return rc;
}

extern "C" int oqp_server_submit(oqp_server* s, const void* packed, uint64_t* ticket)
{
    if (!s || !ticket) return fail(OQP_EINVAL, "oqp_server_submit: NULL argument");
    const PackHdr* h;
    int rc = read_hdr(packed, &h);
    if (rc) return rc;
    if (h->soft && (s->arg.mode != OQP_MODE_F64 || s->arg.ir_max != 0))
        return fail(OQP_EINVAL, "oqp_server_submit: requests with slacks need a server in the FP64 mode without refinement");
    const size_t need = dev_footprint(h);
    if (need > s->arena_bytes) return fail(OQP_ENOMEM, "oqp_server_submit: request needs %zu device bytes, arena %zu",
                                           need, s->arena_bytes);
    size_t off;
    if (s->free_head < 0 || !arena_alloc(s->mem, need, &off)) {
        ++s->rejected;
        return fail(OQP_EBUSY, "oqp_server_submit: no free request slot or device block");
    }
    const int slot = s->free_head;
    Request& r = s->req[slot];
    s->free_head = r.next;
    r.state = RQ_QUEUED;
    ++r.gen;
    r.hdr = h;
    r.dev_off = off;
    r.dev_bytes = need;
    r.group = -1;
    r.next = -1;
    r.tag = 0;
    r.t_submit = now_ns();
    r.t_done = 0;
    r.resume = 0;
    r.iters_done = 0;
    r.ir_done = 0;
    if (s->q_tail < 0) s->q_head = slot; else s->req[s->q_tail].next = slot;
    s->q_tail = slot;
    ++s->queued;
    ++s->submitted;
    *ticket = ((uint64_t)r.gen << 32) | (uint32_t)slot;
    return OQP_OK;
}

// The kernel group of the oldest queued request.  Requests that used up an
// iteration block are queued again at the head, so the head is not always
// the oldest: launching the head's group would let the unfinished requests
// of one group go first round after round while another group's requests
// wait.
static int oldest_variant(const oqp_server* s)
{
    int best = s->q_head;
    for (int r = s->req[best].next; r >= 0; r = s->req[r].next)
        if (s->req[r].t_submit < s->req[best].t_submit) best = r;
    return s->req[best].hdr->variant;
}

extern "C" int oqp_server_progress(oqp_server* s, int* ncompleted)
{
    if (!s) return fail(OQP_EINVAL, "oqp_server_progress: NULL server");
    if (ncompleted) *ncompleted = 0;
    int rc = retire(s, ncompleted);
    if (rc) return rc;
    // launch queued requests on idle streams: the kernel group of the oldest
    // queued request, all of its queued requests up to max_launch (queue
    // order: unfinished requests first)
    while (s->q_head >= 0) {
        const int k = pick_stream(s);
        if (k < 0) break;
        const int gi = free_group(s);
        if (gi < 0) break;
        rc = launch_group(s, s->cfg.iter_block > 0 ? oldest_variant(s) : s->req[s->q_head].hdr->variant, gi, k);
        if (rc) return rc;
    }
    return OQP_OK;
}

extern "C" int oqp_server_poll(const oqp_server* s, uint64_t ticket, oqp_stat* st)
{
    if (!s) return fail(OQP_EINVAL, "oqp_server_poll: NULL server");
    const int slot = ticket_slot(s, ticket);
    if (slot < 0) return fail(OQP_EINVAL, "oqp_server_poll: unknown ticket");
    const Request& r = s->req[slot];
    if (r.state != RQ_DONE) return OQP_PENDING;
    if (st) {
        st->status = r.stat.status;
        st->iters = r.stat.iters;
        st->ir_steps = r.stat.ir_steps;
        st->fell_back_f64 = r.stat.fell_back;
        st->qr_refactors = r.stat.qr_refactors;
        st->mu = r.stat.mu;
        for (int k = 0; k < 4; ++k) st->res[k] = r.stat.res[k];
    }
    return OQP_OK;
}

extern "C" int oqp_server_latency(const oqp_server* s, uint64_t ticket, double* seconds)
{
    if (!s || !seconds) return fail(OQP_EINVAL, "oqp_server_latency: NULL argument");
    const int slot = ticket_slot(s, ticket);
    if (slot < 0) return fail(OQP_EINVAL, "oqp_server_latency: unknown ticket");
    const Request& r = s->req[slot];
    if (r.state != RQ_DONE) return OQP_PENDING;
    *seconds = 1e-9 * (double)(r.t_done - r.t_submit);
    return OQP_OK;
}

extern "C" int oqp_server_get_sol(oqp_server* s, uint64_t ticket, double* u, double* x, double* pi, double* lam_l,
                                  double* lam_u, double* t_l, double* t_u)
{
    if (!s) return fail(OQP_EINVAL, "oqp_server_get_sol: NULL server");
    const int slot = ticket_slot(s, ticket);
    if (slot < 0) return fail(OQP_EINVAL, "oqp_server_get_sol: unknown ticket");
    Request& r = s->req[slot];
    if (r.state != RQ_DONE) return fail(OQP_ESTATE, "oqp_server_get_sol: request not finished");
    const PackHdr* h = r.hdr;
    const size_t bytes = sizeof(double) * h->iter_doubles;
    if (bytes > s->cfg.staging_bytes)
        return fail(OQP_ENOMEM, "oqp_server_get_sol: iterate %zu bytes > staging %zu", bytes, s->cfg.staging_bytes);
    const size_t db = align_up(sizeof(double) * h->data_doubles, 256);
    hipStream_t st = s->streams[0];
    hipError_t e = hipMemcpyAsync(s->staging, s->arena + r.dev_off + db, bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_server_get_sol: %s", hipGetErrorString(e));
    iterate_user_copy((const int*)((const char*)h + h->dims_off), h->N, (const int*)((const char*)h + h->slots_off),
                      oqp::make_layout(h->nx, h->nu, h->ng, h->soft != 0), s->staging, true, u, x, pi, lam_l, lam_u,
                      t_l, t_u);
    return OQP_OK;
}

// Slack blocks of a finished request (after oqp_server_get_sol, from the
// same staged iterate); a request without slacks writes nothing.
extern "C" int oqp_server_get_soft_sol(oqp_server* s, uint64_t ticket, double* s_l, double* s_u, double* lam_sl,
                                       double* lam_su, double* t_sl, double* t_su)
{
    if (!s) return fail(OQP_EINVAL, "oqp_server_get_soft_sol: NULL server");
    const int slot = ticket_slot(s, ticket);
    if (slot < 0) return fail(OQP_EINVAL, "oqp_server_get_soft_sol: unknown ticket");
    Request& r = s->req[slot];
    if (r.state != RQ_DONE) return fail(OQP_ESTATE, "oqp_server_get_soft_sol: request not finished");
    const PackHdr* h = r.hdr;
    if (!h->soft) return OQP_OK;
    const size_t bytes = sizeof(double) * h->iter_doubles;
    if (bytes > s->cfg.staging_bytes)
        return fail(OQP_ENOMEM, "oqp_server_get_soft_sol: iterate %zu bytes > staging %zu", bytes, s->cfg.staging_bytes);
    const size_t db = align_up(sizeof(double) * h->data_doubles, 256);
    hipStream_t st = s->streams[0];
    hipError_t e = hipMemcpyAsync(s->staging, s->arena + r.dev_off + db, bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_server_get_soft_sol: %s", hipGetErrorString(e));
    double* const v[6] = {s_l, s_u, lam_sl, lam_su, t_sl, t_su};
    soft_iterate_copy((const int*)((const char*)h + h->soft_off), h->N, oqp::make_layout(h->nx, h->nu, h->ng, true),
                      s->staging, true, v);
    return OQP_OK;
}

bool server_dims_match(const oqp_server* s, uint64_t ticket, const oqp_dims* d)
{
    const int slot = ticket_slot(s, ticket);
    if (slot < 0) return false;
    const PackHdr* h = s->req[slot].hdr;
    return dims5_match((const int*)((const char*)h + h->dims_off), h->N, d);
}

extern "C" int oqp_server_release(oqp_server* s, uint64_t ticket)
{
    if (!s) return fail(OQP_EINVAL, "oqp_server_release: NULL server");
    const int slot = ticket_slot(s, ticket);
    if (slot < 0) return fail(OQP_EINVAL, "oqp_server_release: unknown ticket");
    Request& r = s->req[slot];
    if (r.state != RQ_DONE) return fail(OQP_ESTATE, "oqp_server_release: request not finished");
    arena_free(s->mem, r.dev_off, r.dev_bytes);
    r.state = RQ_FREE;
    r.hdr = nullptr;
    r.next = s->free_head;
    s->free_head = slot;
    --s->done;
    return OQP_OK;
}

extern "C" int oqp_server_stats(const oqp_server* s, oqp_server_counters* out)
{
    if (!s || !out) return fail(OQP_EINVAL, "oqp_server_stats: NULL argument");
    out->submitted = s->submitted;
    out->rejected = s->rejected;
    out->completed = s->completed;
    out->launches = s->launches;
    out->queued = s->queued;
    out->running = s->running;
    out->done = s->done;
    out->dev_arena = s->arena_bytes;
    out->dev_used = s->mem.used;
    out->dev_peak = s->mem.peak;
    return OQP_OK;
}

extern "C" int oqp_server_replay(oqp_server* s, const void* const* packed, const double* arrival, int count,
                                 double timeout_s, double* latency, oqp_stat* stat, double* wall_s)
{
    if (!s || !packed || !arrival || count < 0 || !latency) return fail(OQP_EINVAL, "oqp_server_replay: bad argument");
    if (s->queued || s->running || s->done) return fail(OQP_ESTATE, "oqp_server_replay: server not idle");
    for (int i = 1; i < count; ++i)
        if (!(arrival[i] >= arrival[i - 1])) return fail(OQP_EINVAL, "oqp_server_replay: arrivals must not decrease");
    for (int i = 0; i < count; ++i) {
        const PackHdr* h;
        int rc = read_hdr(packed[i], &h);
        if (rc) return rc;
        if (dev_footprint(h) > s->arena_bytes) return fail(OQP_ENOMEM, "oqp_server_replay: request %d too large", i);
    }
    s->done_head = s->done_len = 0;
    const int64_t t0 = now_ns();
    int64_t last_event = t0;
    const int64_t limit = (int64_t)(timeout_s * 1e9);
    int next = 0, finished = 0;
    while (finished < count) {
        const int64_t now = now_ns();
        while (next < count && (double)(now - t0) * 1e-9 >= arrival[next]) {
            uint64_t tk;
            int rc = oqp_server_submit(s, packed[next], &tk);
            if (rc == OQP_EBUSY) break;
            if (rc) return rc;
            // latency counts from the scheduled arrival, admission delay included
            Request& r = s->req[(int)(tk & 0xffffffffu)];
            r.tag = next;
            r.t_submit = t0 + (int64_t)(arrival[next] * 1e9);
            ++next;
        }
        int nc = 0;
        int rc = oqp_server_progress(s, &nc);
        if (rc) return rc;
        if (nc) last_event = now_ns();
        while (s->done_len > 0) {
            const int slot = s->done_ring[s->done_head];
            s->done_head = (s->done_head + 1) % s->cfg.max_requests;
            --s->done_len;
            Request& r = s->req[slot];
            const int i = (int)r.tag;
            latency[i] = 1e-9 * (double)(r.t_done - r.t_submit);
            if (stat) {
                oqp_stat& o = stat[i];
                o.status = r.stat.status;
                o.iters = r.stat.iters;
                o.ir_steps = r.stat.ir_steps;
                o.fell_back_f64 = r.stat.fell_back;
                o.qr_refactors = r.stat.qr_refactors;
                o.mu = r.stat.mu;
                for (int k = 0; k < 4; ++k) o.res[k] = r.stat.res[k];
            }
            rc = oqp_server_release(s, ((uint64_t)r.gen << 32) | (uint32_t)slot);
            if (rc) return rc;
            ++finished;
        }
        if (now_ns() - last_event > limit && (s->running > 0 || s->queued > 0))
            return fail(OQP_EDEVICE, "oqp_server_replay: no request finished for %.1f s", timeout_s);
    }
    if (wall_s) *wall_s = 1e-9 * (double)(now_ns() - t0);
    return OQP_OK;
}
