// C-ABI of the gsim library: context, mesh upload, particle state and the
// hot-path entry points. Device memory belongs to the context; host buffers
// are borrowed for the duration of a call. No exception crosses the ABI.
//
// Every hot-path call runs as a batch of surfaces (a single mesh is a batch
// of one): the host prepares each surface's buffers and fills its
// descriptor, the descriptor table goes to device memory when it changed,
// and one binning, one geodesic and one update launch serve the whole
// batch. Steps queue without host synchronisation; several steps can be
// captured once into a HIP graph and replayed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/gsim.h"
#include "gsim_internal.h"

using namespace gsim;

namespace {

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct MeshState {
    HostMesh host;
    DevMesh dm;
    double area = 0.0;  // surface area (computed when first needed)
    // particles
    int n = 0;
    int32_t *face = nullptr;
    double *bary = nullptr, *vel = nullptr, *xyz = nullptr;
    // prefilter
    Buf cell_of, cell_start, cell_fill, order, cand_cnt, cand, tmp64;
    int64_t fill_zero = 0;  // leading cells of cell_fill known to hold zeros
    // candidate-layout results
    Buf cdist, ctan, cflags;
    // pairs
    Buf nbr_cnt, off, nbr, dist, tan, flags;
    int64_t n_pairs = 0;
    // forces / integrator
    Buf F, Ei, E, disp, wflags, step_dev, fire;
    Buf face_nx, bary_nx, vel_nx;  // next state of a fused time step
    uint64_t step = 0;  // steps taken since the state was set: the noise counter (host mirror)
    // all-pairs rows and the particles-by-face index
    int cap = kCandCap;  // row capacity of the last pass
    int ident_n = -1;    // rows hold the identity lists for this n
    Buf fstart, forder, fcount;
};

struct TimingRec {
    double total_ms = 0.0;
    int64_t n = 0;
};

struct GraphRec {
    hipGraphExec_t exec = nullptr;
    int steps = 0;
};

}  // namespace

struct gsim_ctx {
    int device = 0;
    gsim_precision prec = GSIM_FP64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::vector<MeshState *> meshes;
    Buf stack, work, ctr, wstats, scan_scratch, sum_scratch, pf_over, prof, desc, vdist, ttab, roots, partials, vbits;
    Buf gtab;  // big-candidate target arrays of the resident wavefronts
    SurfDesc *desc_pinned = nullptr;  // staging for descriptor uploads
    std::vector<SurfDesc> desc_cached;
    bool profile_sources = false;
    int prof_n = 0;
    int64_t passes = 0;
    GeoParams gp{};
    Counters last{};
    unsigned long long cum_pairs = 0, cum_windows = 0, cum_passes = 0;
    bool timing = false;
    bool time_geodesic_only = false;  // time only the geodesic stage
    bool capturing = false;
    std::map<std::string, TimingRec> times;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> free_events;
    // launch shape
    int max_slots = 65536;
    int lds_stack_kb = 4;
    int grab = 1;
    // the update's wavefronts spread over more compute units (20,000 particles
    // on the height field: 40.4 against 41.7 us with 128, 44.6 with 256)
    int update_block = 64;
    int stack_cap_all = 1 << 18;  // window records per wavefront in all-pairs passes
    double stack_budget = 40e9;   // bytes of window stacks an all-pairs pass may hold
    double table_budget = 96e9;   // bytes of the resident wavefronts' bend-vertex tables
    int max_windows_all = 0;      // per-source window limit in all-pairs passes
    int cus = 256;
    bool whole_mesh = false;  // finite-cutoff passes on the whole-mesh kernel
    int group_sources = 4;  // FP64 persistent passes: sources per wavefront, at most (1, 2 or 4)
    bool fuse_update = true;  // time steps move each particle inside the cutoff kernel
    // layout the bend-vertex tables were last emptied for
    void *roots_p = nullptr;
    int64_t roots_stride = 0;
    int32_t roots_rcap = 0, roots_slots = 0;
    int max_lds = 65536;  // LDS bytes one workgroup may use
    int lds_cu = 163840;  // LDS bytes of one compute unit
    // graphs
    int graph_steps = 50;  // steps captured per graph (0: no graphs)
    std::map<std::string, GraphRec> graphs;
};

// ---- scratch of the allocation-free walk (gsim_displace_on_surface_noalloc)
// One row of 8 walk counts per workgroup of kWalkBlock particles, then the
// 8 totals: 512 KiB, enough for kNoAllocMaxParticles particles. Every GPU the
// library runs on holds its own copy until the process ends. Host code never
// passes the array's name to a kernel (that is a host-side stand-in, not a
// device address): it uses the address hipGetSymbolAddress gave for the
// device, looked up once per device when the first context on it is made.
constexpr int kNoAllocBlocks = 8192;
constexpr int64_t kNoAllocMaxParticles = (int64_t)kNoAllocBlocks * kWalkBlock;  // 2,097,152
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned long long scratch[8 * (kNoAllocBlocks + 1)];
static std::mutex g_scratch_mu;
static unsigned long long *g_scratch[kMaxDevices] = {};

// The device address of `scratch` on `device` (the current device), looked
// up on the first call for that device.
static hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<unsigned long long *>(p);
    return hipSuccess;
}

static unsigned long long *scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[device];
}

namespace {
// Makes the context's device current for one call and gives the caller's
// device back afterwards.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(const gsim_ctx *c) {
        int cur = -1;
        if (c && hipGetDevice(&cur) == hipSuccess && cur != c->device && hipSetDevice(c->device) == hipSuccess)
            prev = cur;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
}  // namespace

namespace {

// Records the message for gsim_last_error. Never throws: a message that
// cannot be stored leaves the error text empty.
gsim_status fail(gsim_ctx *c, gsim_status s, const std::string &msg) noexcept {
    if (c) {
        try {
            c->err = msg;
        } catch (...) {
            c->err.clear();
        }
    }
    return s;
}
gsim_status fail(gsim_ctx *c, gsim_status s, const char *msg) noexcept {
    if (c) {
        try {
            c->err = msg;
        } catch (...) {
            c->err.clear();
        }
    }
    return s;
}

// The handlers that end every entry point's try block: no C++ exception
// crosses the C ABI.
#define GSIM_CATCH(c)                                                     \
    catch (const std::bad_alloc &) {                                      \
        return fail(c, GSIM_E_OOM, "host memory exhausted");              \
    }                                                                     \
    catch (...) {                                                         \
        return fail(c, GSIM_E_ARG, "unexpected host error");              \
    }

#define HIPCHK(c, x)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess)                                                                     \
            return fail(c, e_ == hipErrorOutOfMemory ? GSIM_E_OOM : GSIM_E_DEVICE,                \
                        std::string(#x " failed: ") + hipGetErrorString(e_));                      \
    } while (0)

// Device memory that growing the buffers to the requested sizes takes
// beyond what they hold now (ensure() frees a buffer before it allocates
// 5/4 of the request), checked against what the device has free: an
// oversized request becomes GSIM_E_LIMIT with the byte counts instead of a
// failed allocation halfway through a pass.
struct Grow {
    const Buf *b;
    size_t bytes;
};
gsim_status check_room(gsim_ctx *c, std::initializer_list<Grow> req, const std::string &what) {
    double need = 0.0;
    for (const Grow &g : req)
        if (g.b->bytes < g.bytes) need += 1.25 * (double)g.bytes - (double)g.b->bytes;
    size_t fr = 0, tot = 0;
    if (need <= 0.0 || hipMemGetInfo(&fr, &tot) != hipSuccess) return GSIM_OK;
    if (need <= 0.95 * (double)fr) return GSIM_OK;
    char msg[256];
    std::snprintf(msg, sizeof msg, " need %.3g GB more device memory; %.3g GB of %.3g GB are free", need * 1e-9,
                  (double)fr * 1e-9, (double)tot * 1e-9);
    return fail(c, GSIM_E_LIMIT, what + msg);
}

hipError_t ensure(Buf &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = std::max<size_t>(bytes + bytes / 4, 256);
    hipError_t e = hipMalloc(&b.p, want);
    if (e == hipSuccess) b.bytes = want;
    return e;
}
void release(Buf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}
template <class T>
T *P(Buf &b) {
    return static_cast<T *>(b.p);
}

hipEvent_t take_event(gsim_ctx *c) {
    if (!c->free_events.empty()) {
        hipEvent_t e = c->free_events.back();
        c->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void resolve_timing(gsim_ctx *c) {
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second.second) == hipSuccess &&
            hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            TimingRec &r = c->times[p.first];
            r.total_ms += ms;
            r.n += 1;
        }
        c->free_events.push_back(p.second.first);
        c->free_events.push_back(p.second.second);
    }
    c->pending.clear();
}

// HIP events around one stage, only while timing is on (never inside a
// graph capture). Every event record costs the stream a few microseconds, so
// with `time_geodesic_only` only the geodesic stage is timed.
// A stage of one kernel (`by_kernel`) hands its two events to that kernel's
// launch instead, which has the dispatch itself record them: no extra stream
// commands, and the interval is the kernel's own execution.
struct Stage {
    gsim_ctx *c;
    const char *name;
    bool by_kernel;
    hipEvent_t a = nullptr, b = nullptr;
    Stage(gsim_ctx *c_, const char *n, bool by_kernel_ = false) : c(c_), name(n), by_kernel(by_kernel_) {
        if (c->timing && !c->capturing && (!c->time_geodesic_only || std::strcmp(n, "geodesic") == 0)) {
            a = take_event(c);
            b = take_event(c);
            if (a && !by_kernel) (void)hipEventRecord(a, c->stream);
        }
    }
    ~Stage() {
        if (a && b) {
            if (!by_kernel) (void)hipEventRecord(b, c->stream);
            c->pending.push_back({name, {a, b}});
            if (c->pending.size() > 4096) resolve_timing(c);
        }
    }
};

MeshState *get_mesh(gsim_ctx *c, int32_t id) {
    if (!c || id < 0 || id >= (int32_t)c->meshes.size()) return nullptr;
    return c->meshes[id];
}

bool finite_cutoff(double c) { return c > 0.0 && std::isfinite(c); }
int pot_kind_ok(const gsim_potential *p) { return p && p->kind >= 0 && p->kind <= 2; }

// GSIM_E_NONFINITE when `count` particles met a non-finite value.
gsim_status nonfinite_status(gsim_ctx *c, unsigned long long count) {
    if (!count) return GSIM_OK;
    return fail(c, GSIM_E_NONFINITE,
                std::to_string(count) + " particle(s) met a non-finite force, displacement or velocity and were left "
                                        "in place; gsim_particle_flags marks them (GSIM_PF_NONFINITE)");
}

// ---------------------------------------------------------------- calls
// A call (geodesic_pairs, compute_forces, step) zeroes the device counters,
// queues its work without any host synchronisation, and reads the counters
// back once at the end.
gsim_status begin_call(gsim_ctx *c) {
    HIPCHK(c, launch_zero_u64(P<unsigned long long>(c->ctr), (int64_t)kCtrWords * kCtrSlots * kCtrStride, c->stream));
    HIPCHK(c, launch_zero_i32(P<int32_t>(c->pf_over), 1, c->stream));
    c->passes = 0;
    return GSIM_OK;
}

gsim_status end_call(gsim_ctx *c) {
    int32_t over = 0;
    Counters slots[kCtrSlots * kCtrStride];
    HIPCHK(c, hipMemcpyAsync(slots, c->ctr.p, sizeof(slots), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&over, c->pf_over.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Counters &L = c->last;
    L = Counters{};
    for (int k = 0; k < kCtrSlots; ++k) {
        const Counters &q = slots[k * kCtrStride];
        L.windows += q.windows;
        L.pruned += q.pruned;
        L.launches += q.launches;
        L.stale += q.stale;
        L.guards += q.guards;
        L.nbr_pairs += q.nbr_pairs;
        L.limited += q.limited;
        L.max_depth = std::max(L.max_depth, q.max_depth);
        L.nonfinite += q.nonfinite;
        L.crossings += q.crossings;
    }
    c->cum_pairs += c->last.nbr_pairs;
    c->cum_windows += c->last.windows;
    c->cum_passes += c->passes;
    if (over || c->last.limited)
        return fail(c, GSIM_E_LIMIT,
                    std::to_string(over + (long long)c->last.limited) +
                        " source(s) exceeded a per-source limit (more candidate targets within the cutoff than "
                        "the row capacity set at the start of the call, window stack or window count); the results "
                        "of this call are incomplete. Passes of the whole-mesh kernel (the \"whole_mesh\" knob, up "
                        "to " + std::to_string(kAllPairsMax) + " particles) have no limit on candidates");
    return nonfinite_status(c, c->last.nonfinite);
}

// ---------------------------------------------------------------- batches
// Cell grid of one surface: cells no smaller than the cutoff and at most
// 128 per axis; `small` forces at most kSmallCells cells (one binning
// workgroup per surface) by widening the cells.
void choose_grid(const DevMesh &m, double cutoff, bool small, int dims[3], double &cell) {
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) ext = std::max(ext, m.bbmax[d] - m.bbmin[d]);
    cell = std::max(cutoff, ext / 128.0);
    for (;;) {
        int64_t ncell = 1;
        for (int d = 0; d < 3; ++d) {
            dims[d] = std::max(1, (int)std::ceil((m.bbmax[d] - m.bbmin[d]) / cell));
            ncell *= dims[d];
        }
        if (!small || ncell <= kSmallCells) return;
        cell *= 1.0625;
    }
}

// Surface area of a mesh (computed once).
double surface_area(MeshState *ms) {
    if (!(ms->area > 0.0)) {
        double A = 0.0;
        const HostMesh &H = ms->host;
        for (int f = 0; f < H.nf; ++f) {
            const double *p0 = &H.V[3 * (size_t)H.T[3 * f]], *p1 = &H.V[3 * (size_t)H.T[3 * f + 1]],
                         *p2 = &H.V[3 * (size_t)H.T[3 * f + 2]];
            const double u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
            const double v[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
            const double x = u[1] * v[2] - u[2] * v[1], y = u[2] * v[0] - u[0] * v[2], z = u[0] * v[1] - u[1] * v[0];
            A += 0.5 * std::sqrt(x * x + y * y + z * z);
        }
        ms->area = A;
    }
    return ms->area;
}

// Row capacity of a cutoff pass over the current particle state: kCandCap
// (the LDS target table) while no source can have more Euclidean
// candidates, else the largest count with headroom for the particles' moves
// during the call (the big-candidate kernel). The count runs on the device
// only when the density makes more than kCandCap plausible: three times
// the mean count of a flat disk of radius cutoff.
gsim_status row_capacity(gsim_ctx *c, MeshState *ms, double cutoff, int &cap) {
    const int n = ms->n;
    cap = kCandCap;
    const double mean = n * M_PI * cutoff * cutoff / std::max(surface_area(ms), 1e-300);
    if (3.0 * mean + 16.0 <= kCandCap) return GSIM_OK;
    if (c->capturing) return fail(c, GSIM_E_STATE, "candidate count during graph capture");
    hipStream_t s = c->stream;
    int dims[3];
    double cell;
    choose_grid(ms->dm, cutoff, false, dims, cell);
    const int64_t ncell = (int64_t)dims[0] * dims[1] * dims[2];
    HIPCHK(c, ensure(ms->cell_of, sizeof(int32_t) * n));
    HIPCHK(c, ensure(ms->cell_start, sizeof(int32_t) * (ncell + 1)));
    HIPCHK(c, ensure(ms->cell_fill, sizeof(int32_t) * ncell));
    HIPCHK(c, ensure(ms->order, sizeof(int32_t) * n));
    HIPCHK(c, ensure(ms->tmp64, sizeof(int64_t) * (std::max<int64_t>(ncell, n) + 1)));
    HIPCHK(c, ensure(c->scan_scratch, sizeof(int64_t) * ((std::max<int64_t>(ncell, n) + 1023) / 1024 + 2)));
    HIPCHK(c, ensure(ms->nbr_cnt, sizeof(int32_t) * (n + 1)));
    PrefilterBufs pb{};
    pb.xyz = ms->xyz;
    pb.cell_of = P<int32_t>(ms->cell_of);
    pb.cell_start = P<int32_t>(ms->cell_start);
    pb.cell_fill = P<int32_t>(ms->cell_fill);
    pb.order = P<int32_t>(ms->order);
    pb.cap_c = kCandCap;
    for (int k = 0; k < 3; ++k) pb.dims[k] = dims[k];
    pb.cell = cell;
    HIPCHK(c, launch_cell_sort(ms->dm, n, ms->face, ms->bary, pb, P<int64_t>(c->scan_scratch), true, nullptr,
                               nullptr, false, s));
    ms->fill_zero = ncell;
    HIPCHK(c, launch_count_candidates(n, pb, cutoff * cutoff * (1.0 + 1e-12), P<int32_t>(ms->nbr_cnt), s));
    std::vector<int32_t> cnt(n);
    HIPCHK(c, hipMemcpyAsync(cnt.data(), ms->nbr_cnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const int mx = *std::max_element(cnt.begin(), cnt.end());
    if (mx <= kCandCap) return GSIM_OK;
    if (mx > kBigCandMax)
        return fail(c, GSIM_E_LIMIT, "a source has " + std::to_string(mx) + " Euclidean candidates within the cutoff; "
                                     "the cutoff kernel takes at most " + std::to_string(kBigCandMax) +
                                     " (the \"whole_mesh\" knob has no such limit)");
    cap = std::min(kBigCandMax, (mx + mx / 4 + 32 + 63) / 64 * 64);
    return GSIM_OK;
}

struct Member {
    MeshState *ms;
    double cutoff;
    const gsim_potential *pot;     // may be null (geodesics only)
    const gsim_integrator *integ;  // may be null
};

// Buffers and descriptor of one surface of a batch.
gsim_status prepare_surface(gsim_ctx *c, const Member &mb, bool small, int src_begin, SurfDesc &d) {
    MeshState *ms = mb.ms;
    const int n = ms->n;
    const DevMesh &m = ms->dm;
    if (n <= 0) return fail(c, GSIM_E_STATE, "no particles on this mesh");
    const bool fin = finite_cutoff(mb.cutoff);
    const bool all = !fin || c->whole_mesh;  // rows of every target, whole-mesh kernel
    if (all && n > kAllPairsMax)
        return fail(c, GSIM_E_LIMIT, "whole-mesh passes (no cutoff, or the \"whole_mesh\" knob) hold at most " +
                                         std::to_string(kAllPairsMax) + " particles per surface");
    std::memset(&d, 0, sizeof(d));
    if (all) {
        d.dims[0] = d.dims[1] = d.dims[2] = 1;
        d.cell = 1.0;
    } else {
        choose_grid(m, mb.cutoff, small, d.dims, d.cell);
    }
    const int64_t ncell = (int64_t)d.dims[0] * d.dims[1] * d.dims[2];
    int rowcap = kCandCap;
    if (!all) {
        gsim_status st = row_capacity(c, ms, mb.cutoff, rowcap);
        if (st != GSIM_OK) return st;
    }
    const size_t cap = all ? (size_t)n : (size_t)rowcap;
    if (all) {
        const size_t slots = (size_t)n * cap;
        gsim_status st = check_room(c, {{&ms->cand, 4 * slots}, {&ms->cdist, 8 * slots}, {&ms->ctan, 24 * slots},
                                        {&ms->cflags, slots}},
                                    "the whole-mesh rows of " + std::to_string(n) + " particles (37 bytes a pair slot)");
        if (st != GSIM_OK) return st;
    }
    HIPCHK(c, ensure(ms->cell_of, sizeof(int32_t) * n));
    HIPCHK(c, ensure(ms->cell_start, sizeof(int32_t) * (ncell + 1)));
    {
        const void *was = ms->cell_fill.p;
        HIPCHK(c, ensure(ms->cell_fill, sizeof(int32_t) * ncell));
        if (ms->cell_fill.p != was) ms->fill_zero = 0;  // a new allocation holds no known zeros
    }
    HIPCHK(c, ensure(ms->order, sizeof(int32_t) * n));
    HIPCHK(c, ensure(ms->cand_cnt, sizeof(int32_t) * (n + 1)));
    HIPCHK(c, ensure(ms->cand, sizeof(int32_t) * (size_t)n * cap));
    HIPCHK(c, ensure(ms->cdist, sizeof(double) * (size_t)n * cap));
    HIPCHK(c, ensure(ms->ctan, sizeof(double) * 3 * (size_t)n * cap));
    HIPCHK(c, ensure(ms->cflags, (size_t)n * cap));
    HIPCHK(c, ensure(ms->tmp64, sizeof(int64_t) * (std::max<int64_t>(ncell, n) + 1)));
    HIPCHK(c, ensure(ms->wflags, n));
    const int64_t nscan = std::max<int64_t>(std::max<int64_t>(ncell, n), all ? m.nf : 0);
    HIPCHK(c, ensure(ms->tmp64, sizeof(int64_t) * (nscan + 1)));
    HIPCHK(c, ensure(c->scan_scratch, sizeof(int64_t) * ((nscan + 1023) / 1024 + 2)));
    HIPCHK(c, ensure(ms->F, sizeof(double) * 3 * n));
    HIPCHK(c, ensure(ms->fire, sizeof(FireState)));
    if (all) {
        HIPCHK(c, ensure(ms->fstart, sizeof(int32_t) * (m.nf + 1)));
        HIPCHK(c, ensure(ms->forder, sizeof(int32_t) * n));
        HIPCHK(c, ensure(ms->fcount, sizeof(int32_t) * m.nf));
        if (ms->ident_n != n || ms->cap != (int)cap) {
            HIPCHK(c, launch_identity_rows(n, (int)cap, P<int32_t>(ms->cand_cnt), P<int32_t>(ms->cand), c->stream));
            ms->ident_n = n;
        }
    } else {
        ms->ident_n = -1;  // the candidate search rewrites the rows
    }
    ms->cap = (int)cap;
    d.m = m;
    d.n = n;
    d.src_begin = src_begin;
    d.face = ms->face;
    d.bary = ms->bary;
    d.vel = ms->vel;
    d.xyz = ms->xyz;
    d.cell_of = P<int32_t>(ms->cell_of);
    d.cell_start = P<int32_t>(ms->cell_start);
    d.order = P<int32_t>(ms->order);
    for (int k = 0; k < 3; ++k) d.lo[k] = m.bbmin[k];
    d.cap = (int)cap;
    d.all_pairs = all ? 1 : 0;
    d.fstart = all ? P<int32_t>(ms->fstart) : nullptr;
    d.forder = all ? P<int32_t>(ms->forder) : nullptr;
    d.cand_cnt = P<int32_t>(ms->cand_cnt);
    d.cand = P<int32_t>(ms->cand);
    d.cdist = P<double>(ms->cdist);
    d.ctan = P<double>(ms->ctan);
    d.cflags = P<uint8_t>(ms->cflags);
    d.cutoff = fin ? mb.cutoff : INFINITY;
    d.cut2 = fin ? mb.cutoff * mb.cutoff * (1.0 + 1e-12) : INFINITY;
    if (mb.pot) {
        d.pkind = mb.pot->kind;
        d.pk = mb.pot->k;
        d.psigma = mb.pot->sigma;
    }
    if (mb.integ) {
        d.ikind = mb.integ->kind;
        d.dt = mb.integ->dt;
        d.mobility = mb.integ->mobility;
        d.kT = mb.integ->kT;
        d.friction = mb.integ->friction;
        d.seed = mb.integ->seed;
        const gsim_integrator &g = *mb.integ;
        d.max_disp = g.max_disp > 0.0 ? g.max_disp : INFINITY;
        d.dt_max = g.dt_max > 0.0 ? g.dt_max : 10.0 * g.dt;
        d.alpha0 = g.alpha0 > 0.0 ? g.alpha0 : 0.1;
        d.f_alpha = g.f_alpha > 0.0 ? g.f_alpha : 0.99;
        d.f_inc = g.f_inc > 0.0 ? g.f_inc : 1.1;
        d.f_dec = g.f_dec > 0.0 ? g.f_dec : 0.5;
        d.n_min = g.n_min > 0 ? g.n_min : 5;
    }
    if (!all && mb.integ && mb.integ->kind != GSIM_INT_FIRE) {
        HIPCHK(c, ensure(ms->face_nx, sizeof(int32_t) * n));
        HIPCHK(c, ensure(ms->bary_nx, sizeof(double) * 3 * n));
        HIPCHK(c, ensure(ms->vel_nx, sizeof(double) * 3 * n));
        d.face_out = P<int32_t>(ms->face_nx);
        d.bary_out = P<double>(ms->bary_nx);
        d.vel_out = P<double>(ms->vel_nx);
    }
    d.F = P<double>(ms->F);
    d.fire = P<FireState>(ms->fire);
    d.step = P<uint64_t>(ms->step_dev);
    d.wflags = P<uint8_t>(ms->wflags);
    return GSIM_OK;
}

struct Batch {
    std::vector<Member> mem;
    std::vector<SurfDesc> desc;
    BatchIdx bi{};
    BatchIdx fire_blk{};  // blocks of kFireBlock particles per surface (FIRE reductions)
    bool any_fire = false;
    bool all = false;     // all-pairs surfaces (no cutoff)
    int tcap = 0;         // all-pairs target-table capacity
    int64_t vstride = 0;  // all-pairs vertex-table stride
    int64_t rstride = 0;  // bend-vertex table bytes per wavefront
    int32_t rcap = 0;     // its capacity (bend vertices)
    bool small = true;  // every surface bins in one workgroup
    bool fused = false; // time steps move the particles inside the cutoff kernel
    bool big = false;   // some surface has more candidates per source than the LDS table holds
    int gcap = 0;       // its widest row (big-candidate target arrays per wavefront)
    int group = 1;      // sources per wavefront (FP64, more sources than resident slots: 2 or 4)
    int nslots = 0;
    GeoShape shape{};
};

gsim_status upload_descs(gsim_ctx *c, const std::vector<SurfDesc> &d) {
    const size_t bytes = sizeof(SurfDesc) * d.size();
    if (c->desc_cached.size() == d.size() && std::memcmp(c->desc_cached.data(), d.data(), bytes) == 0)
        return GSIM_OK;
    if (c->capturing) return fail(c, GSIM_E_STATE, "descriptor change during graph capture");
    std::memcpy(c->desc_pinned, d.data(), bytes);
    HIPCHK(c, hipMemcpyAsync(c->desc.p, c->desc_pinned, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->desc_cached = d;
    return GSIM_OK;
}

// Buffers, descriptors and launch shape of a batch.
gsim_status prepare_batch(gsim_ctx *c, Batch &B) {
    const int ns = (int)B.mem.size();
    if (ns < 1 || ns > kMaxBatch) return fail(c, GSIM_E_ARG, "batch size must be 1.." + std::to_string(kMaxBatch));
    for (int i = 0; i < ns; ++i)
        for (int j = 0; j < i; ++j)
            if (B.mem[i].ms == B.mem[j].ms) return fail(c, GSIM_E_ARG, "a mesh appears twice in the batch");
    B.all = !finite_cutoff(B.mem[0].cutoff) || c->whole_mesh;
    for (int i = 1; i < ns; ++i)
        if ((!finite_cutoff(B.mem[i].cutoff) || c->whole_mesh) != B.all)
            return fail(c, GSIM_E_ARG, "a batch mixes cutoff and all-pairs surfaces");
    // a single surface may use the multi-kernel binning for a fine grid
    B.small = true;
    if (ns == 1 && !B.all) {
        int dims[3];
        double cell;
        choose_grid(B.mem[0].ms->dm, B.mem[0].cutoff, false, dims, cell);
        B.small = (int64_t)dims[0] * dims[1] * dims[2] <= kSmallCells;
    }
    B.desc.resize(ns);
    B.bi.nsurf = ns;
    int total = 0;
    for (int i = 0; i < ns; ++i) {
        B.bi.begin[i] = total;
        gsim_status st = prepare_surface(c, B.mem[i], B.small || ns > 1, total, B.desc[i]);
        if (st != GSIM_OK) return st;
        total += B.mem[i].ms->n;
    }
    B.bi.begin[ns] = total;
    B.big = false;
    B.gcap = 0;
    for (int i = 0; i < ns && !B.all; ++i)
        if (B.desc[i].cap > kCandCap) {
            B.big = true;
            B.gcap = std::max(B.gcap, (int)B.desc[i].cap);
        }
    B.fire_blk.nsurf = ns;
    B.any_fire = false;
    int nblk = 0;
    B.tcap = 0;
    B.vstride = 0;
    B.rcap = 1;
    for (int i = 0; i < ns; ++i) {
        B.fire_blk.begin[i] = nblk;
        nblk += (B.mem[i].ms->n + kFireBlock - 1) / kFireBlock;
        B.any_fire |= B.mem[i].integ && B.mem[i].integ->kind == GSIM_INT_FIRE;
        B.tcap = std::max(B.tcap, B.mem[i].ms->n);
        B.vstride = std::max<int64_t>(B.vstride, B.mem[i].ms->dm.nv);
        B.rcap = std::max(B.rcap, B.mem[i].ms->dm.n_pseudo);
    }
    // persistent grid: as many wavefronts as can be resident, at most one per source
    const bool fp32 = c->prec == GSIM_FP32_MIXED;
    const int per_cu = std::max(1, B.all ? geodesic_all_blocks_per_cu(c->lds_stack_kb, fp32)
                                         : geodesic_blocks_per_cu(c->lds_stack_kb, fp32, B.big));
    // several sources per wavefront (the largest group of at most
    // group_sources that still gives every resident wavefront a full one):
    // each of a group's sources has its own bend-vertex entries in the
    // wavefront's table
    B.group = 1;
    if (!B.all && !B.big && !c->profile_sources) {
        // the expected Euclidean candidates of a source (uniform density):
        // a group's sources share the table, so twice that plus 8 must fit a
        // share, or too many sources would run alone (three standard
        // deviations of a Poisson count above the mean: a few in a thousand)
        double mean = 0.0;
        for (int i = 0; i < ns; ++i) {
            const MeshState *ms = B.mem[i].ms;
            const double cut = B.mem[i].cutoff;
            mean = std::max(mean, ms->n * M_PI * cut * cut / std::max(surface_area(B.mem[i].ms), 1e-300));
        }
        // and the resident wavefronts' bend-vertex tables (g entries per
        // bend vertex each) must fit the table budget, or the group would
        // cost resident wavefronts
        const double slots = (double)std::min(c->cus * per_cu, c->max_slots);
        for (int g = c->group_sources; g > 1 && B.group == 1; g /= 2)
            if (total >= (int64_t)g * c->cus * per_cu && mean + 3.0 * std::sqrt(mean) <= (double)(kCandCap / g) &&
                slots * (double)bend_table_bytes(g * B.rcap) <= c->table_budget)
                B.group = g;
    }
    B.rcap *= B.group;
    B.rstride = bend_table_bytes(B.rcap);
    B.fire_blk.begin[ns] = nblk;
    if (B.any_fire) HIPCHK(c, ensure(c->partials, sizeof(double) * 3 * (size_t)std::max(nblk, 1)));
    if (c->profile_sources && ns == 1) {
        const int n = B.mem[0].ms->n;
        if (c->prof_n != n) {
            HIPCHK(c, ensure(c->prof, sizeof(long long) * 8 * (size_t)n));
            HIPCHK(c, launch_zero_u64(P<unsigned long long>(c->prof), 8 * (int64_t)n, c->stream));
            c->prof_n = n;
        }
        B.desc[0].prof = P<long long>(c->prof);
    }
    B.nslots = std::min(std::min(total, c->cus * per_cu), c->max_slots);
    if (B.all) {
        // whole-mesh fronts are deep: fewer resident wavefronts rather than more memory
        const double per_slot = 64.0 * c->stack_cap_all + 8.0 * B.vstride + (double)B.rstride + 32.0 * B.tcap;
        const int64_t fit = (int64_t)(c->stack_budget / per_slot);
        B.nslots = (int)std::max<int64_t>(1, std::min<int64_t>(B.nslots, fit));
    }
    {
        // the bend-vertex tables of the resident wavefronts stay within a budget too
        const int64_t fit = (int64_t)(c->table_budget / (double)std::max<int64_t>(B.rstride, 1));
        B.nslots = (int)std::max<int64_t>(1, std::min<int64_t>(B.nslots, fit));
    }
    // time steps move the particles inside the geodesic launch when there is
    // at most one source per SIMD (four per compute unit): each wavefront's
    // one source then only grows by a walk, and the separate update launch
    // goes. With more sources, every one of them would carry the serial move
    // (measured: a loss from two wavefronts per SIMD on).
    B.fused = c->fuse_update && !B.all && !B.any_fire && total <= B.nslots && total <= 4 * c->cus;
    for (int i = 0; i < ns; ++i) B.fused = B.fused && B.mem[i].integ != nullptr;
    B.shape.lds_stack_kb = c->lds_stack_kb;
    B.shape.nslots = B.nslots;
    B.shape.grab = c->grab;
    B.shape.pad_lds = 0;
    if (!B.all) {
        // fewer sources than resident slots: pad each workgroup's LDS so that
        // at most the needed number fit on a compute unit and the grid spreads
        // over all of them instead of filling some
        const int want = (B.nslots + c->cus - 1) / c->cus;
        const size_t stat = geodesic_lds_bytes(c->lds_stack_kb, fp32, B.big);
        if (want < per_cu && want > 0) {
            const size_t each = (size_t)c->lds_cu / (size_t)want;
            if (each > stat) B.shape.pad_lds = (int32_t)std::min(each - stat, (size_t)c->max_lds - stat);
        }
    }
    const int cap_rec = B.all ? c->stack_cap_all : c->gp.stack_cap;
    HIPCHK(c, ensure(c->stack, (size_t)std::max(B.nslots, 1) * cap_rec * 64));
    if (B.big) HIPCHK(c, ensure(c->gtab, (size_t)std::max(B.nslots, 1) * (size_t)geodesic_gtab_bytes(B.gcap)));
    if (B.all) {
        HIPCHK(c, ensure(c->vdist, sizeof(double) * (size_t)std::max(B.nslots, 1) * B.vstride));
        HIPCHK(c, ensure(c->ttab, 4 * sizeof(double) * (size_t)std::max(B.nslots, 1) * B.tcap));
    }
    // bend-vertex tables: emptied once here, left empty by the kernels
    const int nsl = std::max(B.nslots, 1);
    HIPCHK(c, ensure(c->roots, (size_t)nsl * B.rstride));
    if (c->roots.p != c->roots_p || B.rstride != c->roots_stride || B.rcap != c->roots_rcap ||
        nsl > c->roots_slots) {
        if (c->capturing) return fail(c, GSIM_E_STATE, "bend-vertex tables change during graph capture");
        HIPCHK(c, launch_bend_init(P<char>(c->roots), nsl, B.rstride, B.rcap, c->stream));
        c->roots_p = c->roots.p;
        c->roots_stride = B.rstride;
        c->roots_rcap = B.rcap;
        c->roots_slots = nsl;
    }
    return upload_descs(c, B.desc);
}

const SurfDesc *desc_dev(gsim_ctx *c) { return static_cast<const SurfDesc *>(c->desc.p); }

// Binning, candidate search and geodesics of every source of the batch.
// commit_in: the state to bin is in the next-state arrays (the previous
// fused step of the same call wrote it there).
gsim_status geodesic_pass(gsim_ctx *c, Batch &B, bool advance, bool commit_in = false) {
    hipStream_t s = c->stream;
    if (B.all) {
        {
            Stage st(c, "prefilter");
            HIPCHK(c, launch_pass_begin(desc_dev(c), B.bi.nsurf, P<int32_t>(c->work), advance, s));
            for (size_t i = 0; i < B.mem.size(); ++i) {
                MeshState *ms = B.mem[i].ms;
                HIPCHK(c, launch_face_sort(B.desc[i], P<int32_t>(ms->fcount), P<int64_t>(ms->tmp64),
                                           P<int64_t>(c->scan_scratch), s));
            }
        }
        GeoParams gp = c->gp;
        gp.stack_cap = c->stack_cap_all;
        gp.max_windows = c->max_windows_all;
        Stage st(c, "geodesic");
        HIPCHK(c, launch_geodesic_all(desc_dev(c), B.bi, gp, B.shape, P<char>(c->stack), P<double>(c->vdist), B.vstride,
                                      P<char>(c->roots), B.rstride, B.rcap, P<double2>(c->ttab), B.tcap,
                                      P<int32_t>(c->work), P<Counters>(c->ctr), c->prec == GSIM_FP32_MIXED, s));
        c->passes++;
        return GSIM_OK;
    }
    {
        Stage st(c, "prefilter");
        if (B.small) {
            HIPCHK(c, launch_bin_batch(desc_dev(c), B.bi.nsurf, P<int32_t>(c->work), advance, commit_in, s));
        } else {
            // one surface with a fine grid: multi-kernel counting sort
            MeshState *ms = B.mem[0].ms;
            const SurfDesc &d = B.desc[0];
            const int n = ms->n;
            const int ncell = d.dims[0] * d.dims[1] * d.dims[2];
            PrefilterBufs pb{};
            pb.xyz = ms->xyz;
            pb.cell_of = d.cell_of;
            pb.cell_start = d.cell_start;
            pb.cell_fill = P<int32_t>(ms->cell_fill);
            pb.order = d.order;
            pb.cap_c = kCandCap;
            for (int k = 0; k < 3; ++k) pb.dims[k] = d.dims[k];
            pb.cell = d.cell;
            if (commit_in) HIPCHK(c, launch_commit_batch(desc_dev(c), B.bi, s));
            // starts the pass too (work counters, step counter)
            HIPCHK(c, launch_cell_sort(ms->dm, n, ms->face, ms->bary, pb, P<int64_t>(c->scan_scratch),
                                       ms->fill_zero < ncell, desc_dev(c), P<int32_t>(c->work), advance, s));
            ms->fill_zero = std::max<int64_t>(ms->fill_zero, ncell);
        }
        // several sources per wavefront: their candidate searches run ahead
        // of the pass, at the occupancy of a small kernel
        if (B.group > 1) HIPCHK(c, launch_candidates(desc_dev(c), B.bi, B.group, s));
    }
    GeoParams gp = c->gp;
    if (!(gp.launch_delta > 0.0)) gp.launch_delta = 0.5 * B.mem[0].ms->dm.mean_edge;
    {
        Stage st(c, "geodesic", true);
        HIPCHK(c, launch_geodesic(desc_dev(c), B.bi, gp, B.shape, P<char>(c->stack), P<char>(c->roots), B.rstride,
                                  B.rcap, P<int32_t>(c->work), P<Counters>(c->ctr), c->prec == GSIM_FP32_MIXED,
                                  advance && B.fused, s, st.a, st.b, B.big ? P<char>(c->gtab) : nullptr,
                                  B.big ? B.gcap : 0, B.group, B.group > 1));
    }
    c->passes++;
    return GSIM_OK;
}

gsim_status update_pass(gsim_ctx *c, Batch &B) {
    if (B.fused) return GSIM_OK;  // the particles moved inside the geodesic pass
    if (B.any_fire) {
        Stage sf(c, "fire");
        HIPCHK(c, launch_fire_control(desc_dev(c), B.fire_blk, P<double>(c->partials), P<Counters>(c->ctr), c->stream));
    }
    Stage sg(c, "update");
    HIPCHK(c, launch_update_batch(desc_dev(c), B.bi, c->update_block, P<Counters>(c->ctr), c->stream));
    return GSIM_OK;
}

gsim_status single(gsim_ctx *c, MeshState *ms, double cutoff, const gsim_potential *pot, Batch &B) {
    B.mem.assign(1, Member{ms, cutoff, pot, nullptr});
    gsim_status st = prepare_batch(c, B);
    if (st != GSIM_OK) return st;
    return geodesic_pass(c, B, false);
}

// Compact the candidate rows into the caller-facing CSR (host sync for the size).
gsim_status compact_pairs(gsim_ctx *c, MeshState *ms, double cutoff) {
    hipStream_t s = c->stream;
    const int n = ms->n, cap = ms->cap;
    if (!finite_cutoff(cutoff)) cutoff = INFINITY;
    Stage st(c, "compact");
    HIPCHK(c, ensure(ms->nbr_cnt, sizeof(int32_t) * (n + 1)));
    HIPCHK(c, ensure(ms->off, sizeof(int64_t) * (n + 1)));
    HIPCHK(c, launch_count_rows(n, P<int32_t>(ms->cand_cnt), cap, P<double>(ms->cdist), cutoff,
                                P<int32_t>(ms->nbr_cnt), s));
    HIPCHK(c, launch_scan_i32_to_i64(P<int32_t>(ms->nbr_cnt), P<int64_t>(ms->off), n, P<int64_t>(c->scan_scratch), s));
    int64_t total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, P<int64_t>(ms->off) + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    ms->n_pairs = total;
    {
        const size_t t1 = (size_t)total + 1;
        gsim_status cs = check_room(c, {{&ms->nbr, 4 * t1}, {&ms->dist, 8 * t1}, {&ms->tan, 24 * t1}, {&ms->flags, t1}},
                                    "the " + std::to_string(total) + " pairs of this call (37 bytes each)");
        if (cs != GSIM_OK) return cs;
    }
    HIPCHK(c, ensure(ms->nbr, sizeof(int32_t) * (total + 1)));
    HIPCHK(c, ensure(ms->dist, sizeof(double) * (total + 1)));
    HIPCHK(c, ensure(ms->tan, sizeof(double) * 3 * (total + 1)));
    HIPCHK(c, ensure(ms->flags, total + 1));
    HIPCHK(c, launch_compact_rows(n, P<int32_t>(ms->cand_cnt), cap, P<int32_t>(ms->cand), P<double>(ms->cdist),
                                  P<double>(ms->ctan), P<uint8_t>(ms->cflags), cutoff, P<int64_t>(ms->off),
                                  P<int32_t>(ms->nbr), P<double>(ms->dist), P<double>(ms->tan), P<uint8_t>(ms->flags),
                                  s));
    return GSIM_OK;
}

gsim_status run_forces(gsim_ctx *c, MeshState *ms, const gsim_potential *pot) {
    const int n = ms->n;
    const double cutoff = finite_cutoff(pot->cutoff) ? pot->cutoff : INFINITY;
    HIPCHK(c, ensure(ms->F, sizeof(double) * 3 * n));
    HIPCHK(c, ensure(ms->Ei, sizeof(double) * n));
    HIPCHK(c, ensure(ms->E, sizeof(double) * 4));
    HIPCHK(c, ensure(c->sum_scratch, sizeof(double) * ((n + 255) / 256 + 2)));
    HIPCHK(c, ensure(ms->wflags, n));
    Stage st(c, "forces");
    HIPCHK(c, launch_forces_rows(n, P<int32_t>(ms->cand_cnt), ms->cap, P<double>(ms->cdist), P<double>(ms->ctan),
                                 cutoff, pot->kind, pot->k, pot->sigma, P<double>(ms->F), P<double>(ms->Ei),
                                 &P<Counters>(c->ctr)->nbr_pairs, P<uint8_t>(ms->wflags),
                                 &P<Counters>(c->ctr)->nonfinite, c->stream));
    HIPCHK(c, launch_sum(P<double>(ms->Ei), n, P<double>(ms->E), P<double>(c->sum_scratch), c->stream));
    return GSIM_OK;
}

// Signature of a prepared batch for the graph cache: the descriptor bytes
// (every buffer address and parameter), the kernel parameters and the launch
// shape.
std::string graph_key(gsim_ctx *c, const Batch &B, int steps) {
    std::string k;
    auto put = [&](const void *p, size_t nb) { k.append(static_cast<const char *>(p), nb); };
    put(B.desc.data(), sizeof(SurfDesc) * B.desc.size());
    put(&B.bi, sizeof(B.bi));
    put(&c->gp, sizeof(c->gp));
    put(&B.shape, sizeof(B.shape));
    put(&B.small, sizeof(B.small));
    put(&B.fused, sizeof(B.fused));
    put(&B.big, sizeof(B.big));
    put(&B.group, sizeof(B.group));
    put(&B.gcap, sizeof(B.gcap));
    put(&c->update_block, sizeof(int));
    put(&steps, sizeof(int));
    void *ptrs[10] = {c->stack.p, c->work.p, c->ctr.p, c->desc.p, c->scan_scratch.p, c->vdist.p, c->ttab.p,
                      c->roots.p, c->partials.p, c->gtab.p};
    put(ptrs, sizeof(ptrs));
    const int64_t sizes[4] = {B.rstride, B.rcap, B.tcap, B.vstride};
    put(sizes, sizeof(sizes));
    return k;
}

void drop_graphs(gsim_ctx *c) {
    for (auto &g : c->graphs)
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
    c->graphs.clear();
}

gsim_status enqueue_steps(gsim_ctx *c, Batch &B, int steps) {
    for (int k = 0; k < steps; ++k) {
        gsim_status st = geodesic_pass(c, B, true, B.fused && k > 0);
        if (st != GSIM_OK) return st;
        if ((st = update_pass(c, B)) != GSIM_OK) return st;
    }
    if (B.fused && steps > 0) {
        // the next step's binning commits a fused step's state; after the
        // last one a commit launch does
        Stage sc(c, "commit");
        HIPCHK(c, launch_commit_batch(desc_dev(c), B.bi, c->stream));
    }
    return GSIM_OK;
}

// Run nsteps full steps of a prepared batch: through a cached HIP graph of
// graph_steps steps when timing is off, else eagerly (stage events).
gsim_status run_steps(gsim_ctx *c, Batch &B, int nsteps) {
    gsim_status st;
    const int g = c->graph_steps;
    int done = 0;
    if (!c->timing && g > 0 && nsteps >= 2) {
        const int gs = std::min(g, nsteps);
        const std::string key = graph_key(c, B, gs);
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            if (c->graphs.size() >= 16) drop_graphs(c);
            hipGraph_t graph = nullptr;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            c->capturing = true;
            st = enqueue_steps(c, B, gs);
            c->capturing = false;
            hipError_t e = hipStreamEndCapture(c->stream, &graph);
            if (st != GSIM_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            HIPCHK(c, e);
            GraphRec r;
            r.steps = gs;
            e = hipGraphInstantiate(&r.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPCHK(c, e);
            it = c->graphs.emplace(key, r).first;
            c->passes -= gs;  // the capture counted passes that have not run
        }
        while (nsteps - done >= it->second.steps) {
            HIPCHK(c, hipGraphLaunch(it->second.exec, c->stream));
            done += it->second.steps;
            c->passes += it->second.steps;
        }
    }
    if ((st = enqueue_steps(c, B, nsteps - done)) != GSIM_OK) return st;
    for (auto &m : B.mem) m.ms->step += (uint64_t)nsteps;
    return GSIM_OK;
}

gsim_status check_integ(gsim_ctx *c, const gsim_integrator *integ) {
    if (!integ) return fail(c, GSIM_E_ARG, "null integrator");
    if (integ->kind < GSIM_INT_OVERDAMPED || integ->kind > GSIM_INT_VERLET)
        return fail(c, GSIM_E_ARG, "unknown integrator");
    if (!(integ->dt > 0.0) && integ->kind == GSIM_INT_FIRE) return fail(c, GSIM_E_ARG, "FIRE needs dt > 0");
    return GSIM_OK;
}

template <class T>
hipError_t upload(T *&dst, const T *src, size_t count, hipStream_t s) {
    hipError_t e = hipMalloc(&dst, sizeof(T) * std::max<size_t>(count, 1));
    if (e != hipSuccess) return e;
    if (count) e = hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyHostToDevice, s);
    return e;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

gsim_status gsim_create(int device, gsim_precision prec, void *hip_stream, gsim_ctx **out) {
    if (!out) return GSIM_E_ARG;
    *out = nullptr;
    if (prec != GSIM_FP64 && prec != GSIM_FP32_MIXED) return GSIM_E_ARG;
    gsim_ctx *c = new (std::nothrow) gsim_ctx();
    if (!c) return GSIM_E_OOM;
    c->device = device;
    c->prec = prec;
    if (hipSetDevice(device) != hipSuccess || scratch_setup(device) != hipSuccess) {
        delete c;
        return GSIM_E_DEVICE;
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return GSIM_E_DEVICE;
        }
        c->own_stream = true;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cus = cus;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->max_lds = lds;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) == hipSuccess &&
        lds > 0)
        c->lds_cu = lds;
    // whole-mesh window stacks: at most a quarter of the device's memory
    size_t mem_free = 0, mem_total = 0;
    if (hipMemGetInfo(&mem_free, &mem_total) == hipSuccess && mem_total > 0) {
        c->stack_budget = std::min(c->stack_budget, 0.25 * (double)mem_total);
        // bend-vertex tables: at most a third of it
        c->table_budget = std::min(c->table_budget, (double)mem_total / 3.0);
    }
    c->gp.cutoff = 0.0;
    c->gp.launch_delta = 1e300;  // one bucket: every improved bend vertex once the stack drains
    c->gp.cone_tol = 1e-12;
    c->gp.tie_rel = 1e-9;
    c->gp.guard_rel = 1e-4;
    c->gp.tie_dir = 1e-6;
    c->gp.cone_tol32 = 1e-6;  // 16 times the FP32 rounding of window interval ends
    c->gp.tie_rel32 = 1e-4;
    c->gp.tie_dir32 = 5e-6;
    c->gp.root_rel32 = 2e-6;
    c->gp.slack32 = 1e-4;
    c->gp.bucket = 0.0;
    c->gp.dom_rel = 1e-12;
    c->gp.dom_rel32 = 1e-4;  // FP32 window chains across a whole surface carry errors up to ~1e-5
    c->gp.eager = 0;
    c->gp.stack_cap = 16384;  // 1 MiB of overflow per resident wavefront (wide patches run deep)
    c->gp.max_windows = 4000000;
    c->max_windows_all = 1 << 26;
    if (ensure(c->work, sizeof(int32_t) * kWorkInts) != hipSuccess || ensure(c->ctr, sizeof(Counters) * kCtrSlots * kCtrStride) != hipSuccess ||
        ensure(c->wstats, sizeof(unsigned long long) * 8) != hipSuccess ||
        ensure(c->pf_over, sizeof(int32_t) * 4) != hipSuccess ||
        ensure(c->desc, sizeof(SurfDesc) * kMaxBatch) != hipSuccess ||
        hipHostMalloc((void **)&c->desc_pinned, sizeof(SurfDesc) * kMaxBatch, hipHostMallocDefault) != hipSuccess) {
        gsim_destroy(c);
        return GSIM_E_OOM;
    }
    *out = c;
    return GSIM_OK;
}

void gsim_destroy(gsim_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    try {
        resolve_timing(c);
    } catch (...) {
    }
    drop_graphs(c);
    for (auto e : c->free_events) (void)hipEventDestroy(e);
    for (MeshState *ms : c->meshes) {
        if (!ms) continue;
        for (Buf *b : {&ms->cell_of, &ms->cell_start, &ms->cell_fill, &ms->order, &ms->cand_cnt, &ms->cand,
                       &ms->tmp64, &ms->cdist, &ms->ctan, &ms->cflags, &ms->nbr_cnt, &ms->off, &ms->nbr, &ms->dist,
                       &ms->tan, &ms->flags, &ms->F, &ms->Ei, &ms->E, &ms->disp, &ms->wflags, &ms->step_dev,
                       &ms->fire, &ms->fstart, &ms->forder, &ms->fcount, &ms->face_nx, &ms->bary_nx,
                       &ms->vel_nx})
            release(*b);
        for (void *p : {(void *)ms->face, (void *)ms->bary, (void *)ms->vel, (void *)ms->xyz})
            if (p) (void)hipFree(p);
        for (void *p : {(void *)ms->dm.V, (void *)ms->dm.T, (void *)ms->dm.he, (void *)ms->dm.twin, (void *)ms->dm.hef,
                        (void *)ms->dm.vflag, (void *)ms->dm.theta, (void *)ms->dm.fan_off, (void *)ms->dm.fan,
                        (void *)ms->dm.corner, (void *)ms->dm.fnrm, (void *)ms->dm.fpos,
                        (void *)ms->dm.pidx, (void *)ms->dm.pvert, (void *)ms->dm.prec})
            if (p) (void)hipFree(p);
        delete ms;
    }
    for (Buf *b : {&c->stack, &c->work, &c->ctr, &c->wstats, &c->scan_scratch, &c->sum_scratch, &c->pf_over,
                   &c->prof, &c->desc, &c->vdist, &c->ttab, &c->roots, &c->partials, &c->vbits, &c->gtab})
        release(*b);
    if (c->desc_pinned) (void)hipHostFree(c->desc_pinned);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *gsim_last_error(const gsim_ctx *c) { return c ? c->err.c_str() : "null context"; }

gsim_status gsim_synchronize(gsim_ctx *c) {
    DeviceGuard dg(c);
    try {
        if (!c) return GSIM_E_ARG;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

gsim_status gsim_mesh_upload(gsim_ctx *c, int32_t nv, const double *xyz, int32_t nf, const int32_t *tri,
                             int32_t *mesh_id) {
    DeviceGuard dg(c);
    if (!c || !mesh_id || !xyz || !tri || nv < 3 || nf < 1) return fail(c, GSIM_E_ARG, "bad mesh arguments");
    try {
        MeshState *ms = new MeshState();
        std::string why = build_host_mesh(nv, xyz, nf, tri, ms->host);
        if (!why.empty()) {
            delete ms;
            return fail(c, GSIM_E_MESH, "mesh rejected: " + why);
        }
        HostMesh &H = ms->host;
        DevMesh &d = ms->dm;
        d.nv = nv;
        d.nf = nf;
        hipStream_t s = c->stream;
        // the mesh joins the context first so that a failed copy still frees it
        c->meshes.push_back(ms);
        HIPCHK(c, upload(d.V, H.V.data(), H.V.size(), s));
        HIPCHK(c, upload(d.T, H.T.data(), H.T.size(), s));
        HIPCHK(c, upload(d.he, H.he.data(), H.he.size(), s));
        HIPCHK(c, upload(d.twin, H.twin.data(), H.twin.size(), s));
        HIPCHK(c, upload(d.hef, H.hef.data(), H.hef.size(), s));
        HIPCHK(c, upload(d.vflag, H.vflag.data(), H.vflag.size(), s));
        HIPCHK(c, upload(d.theta, H.theta.data(), H.theta.size(), s));
        HIPCHK(c, upload(d.fan_off, H.fan_off.data(), H.fan_off.size(), s));
        HIPCHK(c, upload(d.fan, H.fan.data(), H.fan.size(), s));
        HIPCHK(c, upload(d.corner, H.corner.data(), H.corner.size(), s));
        HIPCHK(c, upload(d.fnrm, H.fnrm.data(), H.fnrm.size(), s));
        HIPCHK(c, upload(d.fpos, H.fpos.data(), H.fpos.size(), s));
        HIPCHK(c, upload(d.pidx, H.pidx.data(), H.pidx.size(), s));
        HIPCHK(c, upload(d.pvert, H.pvert.data(), H.pvert.size(), s));
        HIPCHK(c, upload(d.prec, H.prec.data(), H.prec.size(), s));
        for (int k = 0; k < 3; ++k) {
            d.bbmin[k] = H.bbmin[k];
            d.bbmax[k] = H.bbmax[k];
        }
        d.mean_edge = H.mean_edge;
        d.min_edge = H.min_edge;
        d.max_edge = H.max_edge;
        d.n_boundary_edges = H.n_boundary_edges;
        d.n_pseudo = H.n_pseudo;
        HIPCHK(c, ensure(ms->step_dev, sizeof(uint64_t)));
        HIPCHK(c, launch_fill_u64(P<unsigned long long>(ms->step_dev), 1, ~0ull, s));
        HIPCHK(c, hipStreamSynchronize(s));
        *mesh_id = (int32_t)c->meshes.size() - 1;
        return GSIM_OK;
    } catch (const std::bad_alloc &) {
        return fail(c, GSIM_E_OOM, "host allocation failed");
    } catch (...) {
        return fail(c, GSIM_E_ARG, "unexpected host error during mesh upload");
    }
}

gsim_status gsim_mesh_info_get(gsim_ctx *c, int32_t id, gsim_mesh_info *out) {
    try {
        MeshState *ms = get_mesh(c, id);
        if (!ms || !out) return fail(c, GSIM_E_ARG, "unknown mesh id");
        const DevMesh &d = ms->dm;
        out->nv = d.nv;
        out->nf = d.nf;
        out->n_boundary_edges = d.n_boundary_edges;
        out->n_pseudo_sources = d.n_pseudo;
        out->mean_edge = d.mean_edge;
        out->min_edge = d.min_edge;
        out->max_edge = d.max_edge;
        for (int k = 0; k < 3; ++k) {
            out->bbox_min[k] = d.bbmin[k];
            out->bbox_max[k] = d.bbmax[k];
        }
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

static gsim_status alloc_particles(gsim_ctx *c, MeshState *ms, int32_t n) {
    if (ms->n == n && ms->face) return GSIM_OK;
    for (void *p : {(void *)ms->face, (void *)ms->bary, (void *)ms->vel, (void *)ms->xyz})
        if (p) (void)hipFree(p);
    ms->face = nullptr;
    ms->bary = ms->vel = ms->xyz = nullptr;
    ms->n = 0;
    HIPCHK(c, hipMalloc(&ms->face, sizeof(int32_t) * std::max(n, 1)));
    HIPCHK(c, hipMalloc(&ms->bary, sizeof(double) * 3 * std::max(n, 1)));
    HIPCHK(c, hipMalloc(&ms->vel, sizeof(double) * 3 * std::max(n, 1)));
    HIPCHK(c, hipMalloc(&ms->xyz, sizeof(double) * 3 * std::max(n, 1)));
    ms->n = n;
    return GSIM_OK;
}

static gsim_status check_state(gsim_ctx *c, const MeshState *ms, int32_t n, const int32_t *face, const double *bary,
                               const double *vel) {
    for (int32_t i = 0; vel && i < 3 * n; ++i)
        if (!std::isfinite(vel[i])) return fail(c, GSIM_E_ARG, "velocity not finite");
    for (int32_t i = 0; i < n; ++i) {
        if (face[i] < 0 || face[i] >= ms->dm.nf) return fail(c, GSIM_E_ARG, "face index out of range");
        const double *b = bary + 3 * (size_t)i;
        int zeros = 0;
        for (int k = 0; k < 3; ++k) {
            if (!(b[k] >= 0.0) || !(b[k] <= 1.0)) return fail(c, GSIM_E_ARG, "barycentric coordinate outside [0,1]");
            zeros += b[k] == 0.0;
        }
        if (std::fabs(b[0] + b[1] + b[2] - 1.0) > 1e-9) return fail(c, GSIM_E_ARG, "barycentric triple must sum to 1");
        if (zeros >= 2) return fail(c, GSIM_E_ARG, "particle placed exactly on a vertex");
    }
    return GSIM_OK;
}

static gsim_status reset_state(gsim_ctx *c, MeshState *ms, const double *vel, hipMemcpyKind kind) {
    hipStream_t s = c->stream;
    const int n = ms->n;
    if (vel) HIPCHK(c, hipMemcpyAsync(ms->vel, vel, sizeof(double) * 3 * n, kind, s));
    else HIPCHK(c, launch_zero_u64(reinterpret_cast<unsigned long long *>(ms->vel), 3 * (int64_t)n, s));
    HIPCHK(c, launch_fill_u64(P<unsigned long long>(ms->step_dev), 1, ~0ull, s));
    HIPCHK(c, ensure(ms->fire, sizeof(FireState)));
    HIPCHK(c, launch_zero_u64(P<unsigned long long>(ms->fire), sizeof(FireState) / 8, s));
    // no flags until a walk, step or force call sets them
    HIPCHK(c, ensure(ms->wflags, (size_t)n + 4));
    HIPCHK(c, launch_zero_i32(P<int32_t>(ms->wflags), (n + 3) / 4, s));
    ms->step = 0;
    return GSIM_OK;
}

gsim_status gsim_particles_set(gsim_ctx *c, int32_t id, int32_t n, const int32_t *face, const double *bary,
                               const double *vel) {
    DeviceGuard dg(c);
    try {
        MeshState *ms = get_mesh(c, id);
        if (!ms || n < 1 || !face || !bary) return fail(c, GSIM_E_ARG, "bad particle arguments");
        gsim_status st = check_state(c, ms, n, face, bary, vel);
        if (st != GSIM_OK) return st;
        if ((st = alloc_particles(c, ms, n)) != GSIM_OK) return st;
        hipStream_t s = c->stream;
        HIPCHK(c, hipMemcpyAsync(ms->face, face, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(ms->bary, bary, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
        if ((st = reset_state(c, ms, vel, hipMemcpyHostToDevice)) != GSIM_OK) return st;
        HIPCHK(c, hipStreamSynchronize(s));
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

gsim_status gsim_particles_set_dev(gsim_ctx *c, int32_t id, int32_t n, const int32_t *face, const double *bary,
                                   const double *vel) {
    DeviceGuard dg(c);
    try {
        MeshState *ms = get_mesh(c, id);
        if (!ms || n < 1 || !face || !bary) return fail(c, GSIM_E_ARG, "bad particle arguments");
        hipStream_t s = c->stream;
        // the same checks as the host path, on the device, before the state is taken
        int32_t *bad = P<int32_t>(c->wstats);
        int32_t hb[3] = {0, 0, 0};
        HIPCHK(c, launch_zero_i32(bad, 3, s));
        HIPCHK(c, launch_validate_state(ms->dm.nf, n, face, bary, vel, bad, s));
        HIPCHK(c, hipMemcpyAsync(hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if (hb[0] || hb[1] || hb[2])
            return fail(c, GSIM_E_ARG, std::to_string(hb[0]) + " face index(es) out of range, " + std::to_string(hb[1]) +
                                           " barycentric triple(s) not in [0,1], not summing to 1 or on a vertex, " +
                                           std::to_string(hb[2]) + " non-finite velocity(ies); state unchanged");
        gsim_status st = alloc_particles(c, ms, n);
        if (st != GSIM_OK) return st;
        HIPCHK(c, hipMemcpyAsync(ms->face, face, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(ms->bary, bary, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
        return reset_state(c, ms, vel, hipMemcpyDeviceToDevice);
    }
    GSIM_CATCH(c)
}

gsim_status gsim_particles_get(gsim_ctx *c, int32_t id, int32_t *face, double *bary, double *vel, double *xyz) {
    DeviceGuard dg(c);
    try {
        MeshState *ms = get_mesh(c, id);
        if (!ms) return fail(c, GSIM_E_ARG, "unknown mesh id");
        if (ms->n <= 0) return fail(c, GSIM_E_STATE, "no particles on this mesh");
        hipStream_t s = c->stream;
        const int n = ms->n;
        if (face) HIPCHK(c, hipMemcpyAsync(face, ms->face, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
        if (bary) HIPCHK(c, hipMemcpyAsync(bary, ms->bary, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
        if (vel) HIPCHK(c, hipMemcpyAsync(vel, ms->vel, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
        if (xyz) {
            HIPCHK(c, launch_xyz(ms->dm, n, ms->face, ms->bary, ms->xyz, s));
            HIPCHK(c, hipMemcpyAsync(xyz, ms->xyz, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
        }
        HIPCHK(c, hipStreamSynchronize(s));
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

gsim_status gsim_particles_get_dev(gsim_ctx *c, int32_t id, int32_t *face, double *bary, double *vel) {
    DeviceGuard dg(c);
    try {
        MeshState *ms = get_mesh(c, id);
        if (!ms) return fail(c, GSIM_E_ARG, "unknown mesh id");
        if (ms->n <= 0) return fail(c, GSIM_E_STATE, "no particles on this mesh");
        hipStream_t s = c->stream;
        const int n = ms->n;
        if (face) HIPCHK(c, hipMemcpyAsync(face, ms->face, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        if (bary) HIPCHK(c, hipMemcpyAsync(bary, ms->bary, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
        if (vel) HIPCHK(c, hipMemcpyAsync(vel, ms->vel, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

// a1-a3 for one surface and the CSR into the caller's buffers (host or
// device memory, by `kind`).
static gsim_status pairs_to(gsim_ctx *c, int32_t id, double cutoff, gsim_pairs *out, hipMemcpyKind kind) {
    DeviceGuard dg(c);
    MeshState *ms = get_mesh(c, id);
    if (!ms || !out) return fail(c, GSIM_E_ARG, "bad arguments");
    try {
        gsim_status st;
        Batch B;
        if ((st = begin_call(c)) != GSIM_OK) return st;
        if ((st = single(c, ms, cutoff, nullptr, B)) != GSIM_OK) return st;
        if ((st = compact_pairs(c, ms, cutoff)) != GSIM_OK) return st;
        if ((st = end_call(c)) != GSIM_OK) return st;
        c->last.nbr_pairs = (unsigned long long)ms->n_pairs;
        c->cum_pairs += c->last.nbr_pairs;
        out->count = ms->n_pairs;
        if (out->capacity < ms->n_pairs || !out->off || (ms->n_pairs && (!out->nbr || !out->dist || !out->tan)))
            return fail(c, GSIM_E_CAPACITY, "pair buffers too small: " + std::to_string(ms->n_pairs) + " needed");
        hipStream_t s = c->stream;
        const int64_t P_ = ms->n_pairs;
        HIPCHK(c, hipMemcpyAsync(out->off, ms->off.p, sizeof(int64_t) * (ms->n + 1), kind, s));
        if (P_) {
            HIPCHK(c, hipMemcpyAsync(out->nbr, ms->nbr.p, sizeof(int32_t) * P_, kind, s));
            HIPCHK(c, hipMemcpyAsync(out->dist, ms->dist.p, sizeof(double) * P_, kind, s));
            HIPCHK(c, hipMemcpyAsync(out->tan, ms->tan.p, sizeof(double) * 3 * P_, kind, s));
            if (out->flags) HIPCHK(c, hipMemcpyAsync(out->flags, ms->flags.p, P_, kind, s));
        }
        if (kind == hipMemcpyDeviceToHost) HIPCHK(c, hipStreamSynchronize(s));
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

gsim_status gsim_geodesic_pairs(gsim_ctx *c, int32_t id, double cutoff, gsim_pairs *out) {
    return pairs_to(c, id, cutoff, out, hipMemcpyDeviceToHost);
}

gsim_status gsim_geodesic_pairs_dev(gsim_ctx *c, int32_t id, double cutoff, gsim_pairs *out) {
    return pairs_to(c, id, cutoff, out, hipMemcpyDeviceToDevice);
}

gsim_status gsim_voronoi_neighbours(gsim_ctx *c, int32_t id, int64_t *off, int32_t *nbr, int64_t capacity,
                                    int64_t *count) {
    DeviceGuard dg(c);
    MeshState *ms = get_mesh(c, id);
    if (!ms || !off || !count) return fail(c, GSIM_E_ARG, "bad arguments");
    const int n = ms->n;
    if (n < 2) return fail(c, GSIM_E_STATE, "fewer than two particles on this mesh");
    if (n > kVoronoiMax)
        return fail(c, GSIM_E_LIMIT, "Voronoi neighbours hold at most " + std::to_string(kVoronoiMax) + " particles");
    try {
        hipStream_t s = c->stream;
        const DevMesh &m = ms->dm;
        surface_area(ms);
        // particle cell grid: cells about one and a half mean spacings wide
        int dims[3];
        double cell;
        choose_grid(m, 1.5 * std::sqrt(ms->area / n), false, dims, cell);
        const int64_t ncell = (int64_t)dims[0] * dims[1] * dims[2];
        HIPCHK(c, ensure(ms->cell_of, sizeof(int32_t) * n));
        HIPCHK(c, ensure(ms->cell_start, sizeof(int32_t) * (ncell + 1)));
        HIPCHK(c, ensure(ms->cell_fill, sizeof(int32_t) * ncell));
        HIPCHK(c, ensure(ms->order, sizeof(int32_t) * n));
        HIPCHK(c, ensure(ms->tmp64, sizeof(int64_t) * (std::max<int64_t>(ncell, n) + 1)));
        HIPCHK(c, ensure(c->scan_scratch, sizeof(int64_t) * ((std::max<int64_t>(ncell, n) + 1023) / 1024 + 2)));
        const int64_t words = (n + 63) / 64;
        HIPCHK(c, ensure(c->vbits, sizeof(unsigned long long) * (size_t)n * words));
        HIPCHK(c, ensure(ms->nbr_cnt, sizeof(int32_t) * (n + 1)));
        HIPCHK(c, ensure(ms->off, sizeof(int64_t) * (n + 1)));
        HIPCHK(c, ensure(c->wstats, sizeof(unsigned long long) * 8));
        PrefilterBufs pb{};
        pb.xyz = ms->xyz;
        pb.cell_of = P<int32_t>(ms->cell_of);
        pb.cell_start = P<int32_t>(ms->cell_start);
        pb.cell_fill = P<int32_t>(ms->cell_fill);
        pb.order = P<int32_t>(ms->order);
        pb.cap_c = kCandCap;
        for (int k = 0; k < 3; ++k) pb.dims[k] = dims[k];
        pb.cell = cell;
        int32_t *err = P<int32_t>(c->wstats);
        {
            Stage st(c, "voronoi");
            HIPCHK(c, launch_cell_sort(m, n, ms->face, ms->bary, pb, P<int64_t>(c->scan_scratch), true, nullptr,
                                       nullptr, false, s));
            ms->fill_zero = ncell;
            HIPCHK(c, launch_zero_u64(P<unsigned long long>(c->vbits), (int64_t)n * words, s));
            HIPCHK(c, launch_zero_i32(err, 2, s));
            HIPCHK(c, launch_voronoi_faces(m, n, ms->xyz, pb.cell_start, pb.order, dims, m.bbmin, cell,
                                           P<unsigned long long>(c->vbits), words, 1e-10 * m.mean_edge, err, s));
            HIPCHK(c, launch_voronoi_count(P<unsigned long long>(c->vbits), n, words, P<int32_t>(ms->nbr_cnt), s));
            HIPCHK(c, launch_scan_i32_to_i64(P<int32_t>(ms->nbr_cnt), P<int64_t>(ms->off), n,
                                             P<int64_t>(c->scan_scratch), s));
        }
        int32_t errs[2] = {0, 0};
        int64_t total = 0;
        HIPCHK(c, hipMemcpyAsync(errs, err, sizeof(errs), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(&total, P<int64_t>(ms->off) + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if (errs[0] || errs[1])
            return fail(c, GSIM_E_LIMIT, std::to_string(errs[0]) + " face(s) with more than 64 candidate particles, " +
                                             std::to_string(errs[1]) + " cell piece(s) with more than 16 vertices");
        *count = total;
        if (capacity < total || (total && !nbr))
            return fail(c, GSIM_E_CAPACITY, "neighbour buffer too small: " + std::to_string(total) + " needed");
        HIPCHK(c, ensure(ms->nbr, sizeof(int32_t) * (total + 1)));
        HIPCHK(c, launch_voronoi_fill(P<unsigned long long>(c->vbits), n, words, P<int64_t>(ms->off), P<int32_t>(ms->nbr),
                                      s));
        HIPCHK(c, hipMemcpyAsync(off, ms->off.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
        if (total) HIPCHK(c, hipMemcpyAsync(nbr, ms->nbr.p, sizeof(int32_t) * total, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return GSIM_OK;
    } catch (...) {
        return fail(c, GSIM_E_ARG, "unexpected host error");
    }
}

// a1-a4 for one surface, the forces and the energy into the caller's
// buffers (host or device memory, by `kind`).
static gsim_status forces_to(gsim_ctx *c, int32_t id, const gsim_potential *pot, double *force, double *energy,
                             hipMemcpyKind kind) {
    DeviceGuard dg(c);
    MeshState *ms = get_mesh(c, id);
    if (!ms || !pot_kind_ok(pot) || !force) return fail(c, GSIM_E_ARG, "bad arguments");
    try {
        gsim_status st;
        Batch B;
        if ((st = begin_call(c)) != GSIM_OK) return st;
        if ((st = single(c, ms, pot->cutoff, pot, B)) != GSIM_OK) return st;
        if ((st = run_forces(c, ms, pot)) != GSIM_OK) return st;
        hipStream_t s = c->stream;
        HIPCHK(c, hipMemcpyAsync(force, ms->F.p, sizeof(double) * 3 * ms->n, kind, s));
        if (energy) HIPCHK(c, hipMemcpyAsync(energy, ms->E.p, sizeof(double), kind, s));
        // the counters are read (a synchronisation) after the copies are queued
        return end_call(c);
    }
    GSIM_CATCH(c)
}

gsim_status gsim_compute_forces(gsim_ctx *c, int32_t id, const gsim_potential *pot, double *force, double *energy) {
    return forces_to(c, id, pot, force, energy, hipMemcpyDeviceToHost);
}

gsim_status gsim_compute_forces_dev(gsim_ctx *c, int32_t id, const gsim_potential *pot, double *force,
                                    double *energy) {
    return forces_to(c, id, pot, force, energy, hipMemcpyDeviceToDevice);
}

// The walk of every particle by disp (device memory) and its statistics.
static gsim_status walk_dev(gsim_ctx *c, MeshState *ms, const double *disp, int transport_velocity,
                            gsim_walk_stats *stats) {
    const int n = ms->n;
    hipStream_t s = c->stream;
    HIPCHK(c, ensure(ms->wflags, n));
    HIPCHK(c, launch_zero_u64(P<unsigned long long>(c->wstats), 8, s));
    {
        Stage st(c, "walk");
        HIPCHK(c, launch_walk(ms->dm, n, ms->face, ms->bary, disp, transport_velocity ? ms->vel : nullptr,
                              P<unsigned long long>(c->wstats), P<uint8_t>(ms->wflags), s));
    }
    unsigned long long h[8];
    HIPCHK(c, hipMemcpyAsync(h, c->wstats.p, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (stats) {
        stats->crossings = (int64_t)h[0];
        stats->vertex_hits = (int64_t)h[1];
        stats->boundary_hits = (int64_t)h[2];
        stats->cap_hits = (int64_t)h[3];
        stats->near_vertex = (int64_t)h[4];
        stats->nonfinite = (int64_t)h[5];
    }
    return nonfinite_status(c, h[5]);
}

gsim_status gsim_displace_on_surface(gsim_ctx *c, int32_t id, const double *disp, int transport_velocity,
                                     gsim_walk_stats *stats) {
    DeviceGuard dg(c);
    MeshState *ms = get_mesh(c, id);
    if (!ms || !disp) return fail(c, GSIM_E_ARG, "bad arguments");
    if (ms->n <= 0) return fail(c, GSIM_E_STATE, "no particles on this mesh");
    try {
        HIPCHK(c, ensure(ms->disp, sizeof(double) * 3 * ms->n));
        HIPCHK(c, hipMemcpyAsync(ms->disp.p, disp, sizeof(double) * 3 * ms->n, hipMemcpyHostToDevice, c->stream));
        return walk_dev(c, ms, P<double>(ms->disp), transport_velocity, stats);
    }
    GSIM_CATCH(c)
}

gsim_status gsim_displace_on_surface_dev(gsim_ctx *c, int32_t id, const double *disp, int transport_velocity,
                                         gsim_walk_stats *stats) {
    DeviceGuard dg(c);
    MeshState *ms = get_mesh(c, id);
    if (!ms || !disp) return fail(c, GSIM_E_ARG, "bad arguments");
    if (ms->n <= 0) return fail(c, GSIM_E_STATE, "no particles on this mesh");
    try {
        return walk_dev(c, ms, disp, transport_velocity, stats);
    }
    GSIM_CATCH(c)
}

gsim_status gsim_displace_on_surface_noalloc(gsim_ctx *c, int32_t id, const double *disp, int transport_velocity,
                                             uint8_t *flags, gsim_walk_stats *stats) {
    DeviceGuard dg(c);
    MeshState *ms = get_mesh(c, id);
    if (!ms || !disp) return fail(c, GSIM_E_ARG, "bad arguments");
    if (ms->n <= 0) return fail(c, GSIM_E_STATE, "no particles on this mesh");
    if (ms->n > kNoAllocMaxParticles)
        return fail(c, GSIM_E_LIMIT, "the allocation-free walk takes at most " + std::to_string(kNoAllocMaxParticles) +
                                         " particles per call (" + std::to_string(ms->n) + " on this mesh)");
    unsigned long long *part = scratch_of(c->device);
    if (!part) return fail(c, GSIM_E_STATE, "walk scratch not set up on this device");
    try {
        // no allocation: the context's particle state, the caller's buffers
        // and the device's scratch array only; every row of the scratch the
        // kernels read is written by this call first
        hipStream_t s = c->stream;
        unsigned long long *tot = part + 8 * (int64_t)kNoAllocBlocks;
        HIPCHK(c, launch_walk_blocks(ms->dm, ms->n, ms->face, ms->bary, disp, transport_velocity ? ms->vel : nullptr,
                                     flags, part, tot, s));
        unsigned long long h[8];
        HIPCHK(c, hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if (stats) {
            stats->crossings = (int64_t)h[0];
            stats->vertex_hits = (int64_t)h[1];
            stats->boundary_hits = (int64_t)h[2];
            stats->cap_hits = (int64_t)h[3];
            stats->near_vertex = (int64_t)h[4];
            stats->nonfinite = (int64_t)h[5];
        }
        return nonfinite_status(c, h[5]);
    }
    GSIM_CATCH(c)
}

// Per-particle flags of the last walk, step or force call on the mesh
// (host or device buffer, by `kind`).
static gsim_status flags_to(gsim_ctx *c, int32_t id, uint8_t *flags, hipMemcpyKind kind) {
    DeviceGuard dg(c);
    MeshState *ms = get_mesh(c, id);
    if (!ms || !flags) return fail(c, GSIM_E_ARG, "bad arguments");
    if (ms->n <= 0) return fail(c, GSIM_E_STATE, "no particles on this mesh");
    try {
        hipStream_t s = c->stream;
        HIPCHK(c, hipMemcpyAsync(flags, ms->wflags.p, ms->n, kind, s));
        if (kind == hipMemcpyDeviceToHost) HIPCHK(c, hipStreamSynchronize(s));
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

gsim_status gsim_particle_flags(gsim_ctx *c, int32_t id, uint8_t *flags) {
    return flags_to(c, id, flags, hipMemcpyDeviceToHost);
}

gsim_status gsim_particle_flags_dev(gsim_ctx *c, int32_t id, uint8_t *flags) {
    return flags_to(c, id, flags, hipMemcpyDeviceToDevice);
}

gsim_status gsim_step_batched(gsim_ctx *c, int32_t nmesh, const int32_t *mesh_ids, const gsim_potential *pots,
                              const gsim_integrator *integs, int32_t nsteps) {
    DeviceGuard dg(c);
    if (!c || nmesh < 1 || nmesh > kMaxBatch || !mesh_ids || !pots || !integs || nsteps < 0)
        return fail(c, GSIM_E_ARG, "bad arguments");
    try {
        Batch B;
        for (int32_t i = 0; i < nmesh; ++i) {
            MeshState *ms = get_mesh(c, mesh_ids[i]);
            if (!ms) return fail(c, GSIM_E_ARG, "unknown mesh id in batch");
            if (!pot_kind_ok(&pots[i])) return fail(c, GSIM_E_ARG, "unknown potential in batch");
            gsim_status st = check_integ(c, &integs[i]);
            if (st != GSIM_OK) return st;
            B.mem.push_back(Member{ms, pots[i].cutoff, &pots[i], &integs[i]});
        }
        gsim_status st;
        if ((st = begin_call(c)) != GSIM_OK) return st;
        if ((st = prepare_batch(c, B)) != GSIM_OK) return st;
        if ((st = run_steps(c, B, nsteps)) != GSIM_OK) return st;
        return end_call(c);
    } catch (...) {
        return fail(c, GSIM_E_ARG, "unexpected host error");
    }
}

gsim_status gsim_step(gsim_ctx *c, int32_t id, const gsim_potential *pot, const gsim_integrator *integ,
                      int32_t nsteps) {
    DeviceGuard dg(c);
    if (!get_mesh(c, id)) return fail(c, GSIM_E_ARG, "unknown mesh id");
    return gsim_step_batched(c, 1, &id, pot, integ, nsteps);
}

gsim_status gsim_autotune(gsim_ctx *c, int32_t nmesh, const int32_t *mesh_ids, const gsim_potential *pots,
                          const gsim_integrator *integs, int32_t reps, double *out) {
    DeviceGuard dg(c);
    if (!c || nmesh < 1 || nmesh > kMaxBatch || !mesh_ids || !pots || !integs || reps < 1)
        return fail(c, GSIM_E_ARG, "bad arguments");
    try {
        Batch B;
        for (int32_t i = 0; i < nmesh; ++i) {
            MeshState *ms = get_mesh(c, mesh_ids[i]);
            if (!ms || !pot_kind_ok(&pots[i])) return fail(c, GSIM_E_ARG, "bad batch member");
            gsim_status st = check_integ(c, &integs[i]);
            if (st != GSIM_OK) return st;
            B.mem.push_back(Member{ms, pots[i].cutoff, &pots[i], &integs[i]});
        }
        const bool was_timing = c->timing;
        c->timing = false;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        struct Cand {
            int kb, grab;
        };
        const Cand cands[] = {{16, 1}, {8, 1}, {4, 1}, {16, 2}, {8, 2}, {4, 2}, {8, 4}, {4, 4}};
        double best = INFINITY;
        Cand pick = {c->lds_stack_kb, c->grab};
        gsim_status st = GSIM_OK;
        for (const Cand &k : cands) {
            c->lds_stack_kb = k.kb;
            c->grab = k.grab;
            if ((st = begin_call(c)) != GSIM_OK) break;
            if ((st = prepare_batch(c, B)) != GSIM_OK) break;
            if ((st = geodesic_pass(c, B, false)) != GSIM_OK) break;  // warm-up
            double tmin = INFINITY;
            for (int r = 0; r < reps && st == GSIM_OK; ++r) {
                float ms = 0.f;
                hipError_t e = hipEventRecord(e0, c->stream);
                if (e == hipSuccess) st = geodesic_pass(c, B, false);
                if (e == hipSuccess && st == GSIM_OK) e = hipEventRecord(e1, c->stream);
                if (e == hipSuccess && st == GSIM_OK) e = hipEventSynchronize(e1);
                if (e == hipSuccess && st == GSIM_OK) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) st = fail(c, GSIM_E_DEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
                tmin = std::min(tmin, (double)ms);
            }
            if (st != GSIM_OK) break;
            if ((st = end_call(c)) != GSIM_OK) break;
            if (tmin < best) {
                best = tmin;
                pick = k;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c->lds_stack_kb = pick.kb;
        c->grab = pick.grab;
        c->timing = was_timing;
        if (st != GSIM_OK) return st;
        // update workgroup size: timed on a scratch copy of the particle
        // state (the rows of the last geodesic pass stay valid for it)
        int best_block = c->update_block;
        {
            if ((st = prepare_batch(c, B)) != GSIM_OK) return st;
            std::vector<SurfDesc> scratch = B.desc;
            std::vector<Buf> bufs;
            auto cleanup = [&]() {
                (void)hipStreamSynchronize(c->stream);
                for (auto &b : bufs) release(b);
            };
            for (auto &d : scratch) {
                Buf f, b, v, s, w;
                if (ensure(f, sizeof(int32_t) * d.n) != hipSuccess || ensure(b, sizeof(double) * 3 * d.n) != hipSuccess ||
                    ensure(v, sizeof(double) * 3 * d.n) != hipSuccess || ensure(s, sizeof(uint64_t)) != hipSuccess ||
                    ensure(w, d.n) != hipSuccess) {
                    for (Buf *x : {&f, &b, &v, &s, &w}) bufs.push_back(*x);
                    cleanup();
                    return fail(c, GSIM_E_OOM, "autotune scratch allocation failed");
                }
                (void)hipMemcpyAsync(f.p, d.face, sizeof(int32_t) * d.n, hipMemcpyDeviceToDevice, c->stream);
                (void)hipMemcpyAsync(b.p, d.bary, sizeof(double) * 3 * d.n, hipMemcpyDeviceToDevice, c->stream);
                (void)hipMemcpyAsync(v.p, d.vel, sizeof(double) * 3 * d.n, hipMemcpyDeviceToDevice, c->stream);
                (void)launch_zero_u64(P<unsigned long long>(s), 1, c->stream);
                d.face = P<int32_t>(f);
                d.bary = P<double>(b);
                d.vel = P<double>(v);
                d.step = P<uint64_t>(s);
                d.wflags = P<uint8_t>(w);
                for (Buf *x : {&f, &b, &v, &s, &w}) bufs.push_back(*x);
            }
            if ((st = upload_descs(c, scratch)) != GSIM_OK) {
                cleanup();
                return st;
            }
            hipEvent_t a0 = nullptr, a1 = nullptr;
            (void)hipEventCreate(&a0);
            (void)hipEventCreate(&a1);
            double bt = INFINITY;
            for (int blk : {64, 128, 256}) {
                double tmin = INFINITY;
                for (int r = 0; r < reps + 1; ++r) {
                    float ms = 0.f;
                    (void)hipEventRecord(a0, c->stream);
                    (void)launch_update_batch(desc_dev(c), B.bi, blk, P<Counters>(c->ctr), c->stream);
                    (void)hipEventRecord(a1, c->stream);
                    if (hipEventSynchronize(a1) == hipSuccess && hipEventElapsedTime(&ms, a0, a1) == hipSuccess && r > 0)
                        tmin = std::min(tmin, (double)ms);
                }
                if (tmin < bt) {
                    bt = tmin;
                    best_block = blk;
                }
            }
            (void)hipEventDestroy(a0);
            (void)hipEventDestroy(a1);
            cleanup();
            c->desc_cached.clear();  // the table on the device holds the scratch descriptors
        }
        c->update_block = best_block;
        drop_graphs(c);
        if (out) {
            out[0] = c->lds_stack_kb;
            out[1] = c->grab;
            out[2] = c->update_block;
            out[3] = best;
        }
        return GSIM_OK;
    } catch (...) {
        return fail(c, GSIM_E_ARG, "unexpected host error");
    }
}

gsim_status gsim_timing_enable(gsim_ctx *c, int on) {
    DeviceGuard dg(c);
    try {
        if (!c) return GSIM_E_ARG;
        resolve_timing(c);
        c->timing = on != 0;
        if (on) {
            c->times.clear();
            c->cum_pairs = c->cum_windows = c->cum_passes = 0;
        }
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

gsim_status gsim_timing_get(gsim_ctx *c, const char *name, double *avg_ms, int64_t *launches) {
    DeviceGuard dg(c);
    try {
        if (!c || !name) return GSIM_E_ARG;
        resolve_timing(c);
        auto it = c->times.find(name);
        if (it == c->times.end()) {
            if (avg_ms) *avg_ms = 0.0;
            if (launches) *launches = 0;
            return GSIM_OK;
        }
        if (avg_ms) *avg_ms = it->second.n ? it->second.total_ms / double(it->second.n) : 0.0;
        if (launches) *launches = it->second.n;
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

gsim_status gsim_tune_set(gsim_ctx *c, const char *name, double value) {
    DeviceGuard dg(c);
    try {
        if (!c || !name) return GSIM_E_ARG;
        std::string k(name);
        if (k == "launch_delta") c->gp.launch_delta = value;
        else if (k == "cone_tol" && value >= 0.0) c->gp.cone_tol = value;
        else if (k == "tie_rel" && value >= 0.0) c->gp.tie_rel = value;
        else if (k == "tie_dir" && value >= 0.0) c->gp.tie_dir = value;
        else if (k == "eager") c->gp.eager = value != 0.0;
        else if (k == "cone_tol32" && value >= 0.0) c->gp.cone_tol32 = value;
        else if (k == "tie_rel32" && value >= 0.0) c->gp.tie_rel32 = value;
        else if (k == "tie_dir32" && value >= 0.0) c->gp.tie_dir32 = value;
        else if (k == "guard_rel" && value >= 0.0) c->gp.guard_rel = value;
        else if (k == "root_rel32" && value >= 0.0 && value <= 1e-4) c->gp.root_rel32 = value;
        else if (k == "slack32" && value >= 1e-6 && value <= 1e-2) c->gp.slack32 = value;
        else if (k == "stack_cap" && value >= 64 && value <= (1 << 22)) c->gp.stack_cap = (int32_t)value;
        else if (k == "max_windows" && value >= 1) c->gp.max_windows = (int32_t)std::min(value, 2.0e9);
        else if (k == "max_slots" && value >= 1 && value <= 65536) c->max_slots = (int)value;
        else if (k == "lds_stack_kb" && (value == 4 || value == 8 || value == 16)) c->lds_stack_kb = (int)value;
        else if (k == "grab" && value >= 1 && value <= 64) c->grab = (int)value;
        else if (k == "update_block" && (value == 64 || value == 128 || value == 256)) c->update_block = (int)value;
        else if (k == "graph_steps" && value >= 0 && value <= 1000) c->graph_steps = (int)value;
        else if (k == "stack_cap_all" && value >= 1024 && value <= (1 << 22)) c->stack_cap_all = (int)value;
        else if (k == "max_windows_all" && value >= 1) c->max_windows_all = (int32_t)std::min(value, 2.0e9);
        else if (k == "bucket" && value >= 0.0) c->gp.bucket = value;
        else if (k == "dom_rel" && value >= 0.0) c->gp.dom_rel = value;
        else if (k == "dom_rel32" && value >= 0.0) c->gp.dom_rel32 = value;
        else if (k == "whole_mesh" && (value == 0.0 || value == 1.0)) c->whole_mesh = value != 0.0;
        else if (k == "group_sources" && (value == 1.0 || value == 2.0 || value == 4.0 || value == 8.0))
            c->group_sources = (int)value;
        else if (k == "fuse_update" && (value == 0.0 || value == 1.0)) c->fuse_update = value != 0.0;
        else if (k == "time_geodesic_only" && (value == 0.0 || value == 1.0)) c->time_geodesic_only = value != 0.0;
        else return fail(c, GSIM_E_ARG, "unknown tuning knob or value out of range: " + k);
        drop_graphs(c);
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

gsim_status gsim_source_profile(gsim_ctx *c, int on, int64_t *out, int32_t n) {
    DeviceGuard dg(c);
    try {
        if (!c) return GSIM_E_ARG;
        if (out) {
            if (!c->profile_sources || n != c->prof_n) return fail(c, GSIM_E_STATE, "source profiling not active");
            HIPCHK(c, hipMemcpyAsync(out, c->prof.p, sizeof(long long) * 8 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        c->profile_sources = on != 0;
        c->prof_n = 0;
        return GSIM_OK;
    }
    GSIM_CATCH(c)
}

gsim_status gsim_counters_get(gsim_ctx *c, int64_t *c10) {
    if (!c || !c10) return GSIM_E_ARG;
    c10[12] = (int64_t)c->last.crossings;
    c10[11] = (int64_t)c->last.nonfinite;
    c10[10] = (int64_t)c->last.max_depth;
    c10[7] = (int64_t)c->cum_pairs;
    c10[8] = (int64_t)c->cum_windows;
    c10[9] = (int64_t)c->cum_passes;
    c10[0] = (int64_t)c->last.windows;
    c10[1] = (int64_t)c->last.pruned;
    c10[2] = (int64_t)c->last.launches;
    c10[3] = (int64_t)c->last.stale;
    c10[4] = (int64_t)c->last.guards;
    c10[5] = (int64_t)c->last.nbr_pairs;
    c10[6] = (int64_t)c->last.limited;
    return GSIM_OK;
}

}  // extern "C"
