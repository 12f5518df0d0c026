// Solver driver and C ABI (include/mg.h).
//
// Outer loop (paper Section 2: each iteration reduces ||b - Hu||): in FP64,
//   r = b - H u;  while ||r|| > tol ||b||:  e = V(r);  u += e;  r = b - H u
// with the V-cycle V in FP32 (mixed) or FP64. The update, the residual and its
// norm are one fused FP64 kernel; the norm is the only per-iteration
// device-to-host transfer (8 bytes).
//
// V-cycle on level l with right-hand side f (Sections 2, 2.1, 2.3):
//   x = omega H_z^{-1} f; (nu_pre - 1) more sweeps;
//   f_{l+1} = R (f - H x); x_{l+1} = V_{l+1}(f_{l+1}); x += P x_{l+1};
//   nu_post sweeps; the coarsest level does coarse_sweeps sweeps from zero.
// The transposed V-cycle (adjoint solve) is the transpose of that map f -> x.
// H and every H_z are symmetric, so the transpose of a chain of sweeps from
// zero is the chain of the same sweeps in reverse order from zero, and the
// transposed cycle has the forward cycle's shape: nu_post sweeps with the
// post-smoothing factors reversed; f_{l+1} = P^T (f - H x); the transposed
// coarse cycle; x += R^T x_{l+1}; nu_pre sweeps with the pre-smoothing
// factors reversed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "mg.h"
#include "setup.hpp"

namespace {

template <typename T>
struct Work {
    T* f = nullptr;     // right-hand side of the level
    T* xa = nullptr;    // iterate (ping)
    T* xb = nullptr;    // iterate (pong)
};

struct DevLevel {
    int nI = 0, nJ = 0, nz = 0;
    long long plane = 0, n = 0;
    double *Tlam64 = nullptr, *Tth64 = nullptr, *Tr64 = nullptr, *V64 = nullptr;
    float *Tlam32 = nullptr, *Tth32 = nullptr, *Tr32 = nullptr;
    double *M64 = nullptr, *invp64 = nullptr;
    float *M32 = nullptr, *invp32 = nullptr;
    mgk::StepCoef<double>* sc64 = nullptr;
    mgk::StepCoef<float>* sc32 = nullptr;
    // to the next coarser level
    int *crow_of = nullptr, *prow = nullptr;
    double* pw64 = nullptr;
    float* pw32 = nullptr;
    // from the next finer level
    int *child_first = nullptr, *child_count = nullptr, *ptrow = nullptr;
    double* ptw64 = nullptr;
    float* ptw32 = nullptr;
    Work<float> w32;
    Work<double> w64;
};

struct ProfRec {
    int cls, level;
    double bytes;
    hipEvent_t a, b;
    int launches = 1;   // consecutive launches of class cls between a and b
};

// Explicit matrix C of the coarsest-level solve (x = C f), and C^T for the
// transposed cycle, in both precisions; formed for the current coefficients,
// omega and number of sweeps.
struct DenseCoarse {
    bool enabled = false;   // the coarsest level is small enough
    bool valid = false;     // matrices match the current coefficients/options
    long long n = 0;
    int sweeps = -1;
    double omega = 0;
    double *C64 = nullptr, *Ct64 = nullptr;
    float *C32 = nullptr, *Ct32 = nullptr;
};

}  // namespace

struct mg_handle {
    mg_grid grid{};
    mg_options opt{};
    mgs::Hierarchy host;
    std::vector<DevLevel> lv;
    hipStream_t stream = nullptr;
    std::vector<void*> allocs;
    double* u_alt = nullptr;       // FP64 iterate buffers beside the caller's u
    double* u_alt2 = nullptr;
    float *u32a = nullptr, *u32b = nullptr, *b32 = nullptr;   // MG_PREC_FP32 solve
    double* partials = nullptr;
    double* scalar = nullptr;      // device: reduced values [2]
    double* host_scalar = nullptr; // pinned host copy [2]
    hipEvent_t scalar_ready = nullptr;   // recorded after the copy to host_scalar
    int max_partials = 0;
    size_t max_lds = 64 * 1024;    // LDS bytes a block may use (device limit)
    int device = 0;                // the GPU the handle lives on
    bool no_events = false;        // record no HIP events (mg_solve_noalloc)
    bool have32 = false, have64 = false;
    DenseCoarse dense;
    // The V-cycle below the finest level (levels 1..L-1), per precision,
    // captured once as a HIP graph and replayed in every forward cycle.
    struct CoarseGraph {
        hipGraphExec_t exec = nullptr;
        void* result = nullptr;       // the level-1 buffer the cycle leaves its result in
        double bytes = 0;             // its algorithmic bytes
        bool dense_valid = false;     // the coarsest route it was captured with
    } g32, g64;
    hipStream_t cap_stream = nullptr; // private stream the graphs are captured on
    bool capturing = false;
    bool no_graphs = false;           // replay none (mg_solve_noalloc)
    bool log = false;                 // MG_LOG set at setup: one line per iteration
    std::string err;
    std::vector<ProfRec> recs;
    std::vector<ProfRec> phases;   // cls 0: a V-cycle, 1: a refinement step
    std::vector<hipEvent_t> events;
    size_t next_event = 0;
    double alg_bytes = 0;
};

namespace {

mg_status fail(mg_handle* h, mg_status s, const char* fmt, ...) {
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->err = buf;
    }
    return s;
}

#define HIP_TRY(h, call)                                                              \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail((h), MG_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define MG_TRY(call)                   \
    do {                               \
        mg_status s_ = (call);         \
        if (s_ != MG_OK) return s_;    \
    } while (0)

mg_status check_launch(mg_handle* h, const char* what);

template <typename T>
mg_status dalloc(mg_handle* h, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, MG_ERR_OOM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                    hipGetErrorString(e));
    }
    h->allocs.push_back(q);
    *p = static_cast<T*>(q);
    // poison: floating-point arrays start as quiet NaN (ordered before any
    // upload or kernel on the handle's stream), so that a result depending
    // on memory the library never wrote shows as NaN
    if constexpr (std::is_same<T, float>::value || std::is_same<T, double>::value) {
        if (h->opt.poison) {
            mgk::fill<T>(*p, std::numeric_limits<T>::quiet_NaN(), (long long)count, h->stream);
            MG_TRY(check_launch(h, "fill"));
        }
    }
    return MG_OK;
}

// The step records of a level's column sweeps (mgk::StepCoef): for each
// direction and row, the couplings of the layers in the order a wavefront
// of a twisted pair walks them.
template <typename T>
std::vector<mgk::StepCoef<T>> step_table(const mgs::Level& s) {
    const int nJ = s.nJ, nz = s.nz;
    std::vector<mgk::StepCoef<T>> tab(size_t(2) * nJ * mgk::kStepStride);
    for (int dir = 0; dir < 2; ++dir)
        for (int J = 0; J < nJ; ++J)
            for (int t = 0; t < mgk::kStepStride; ++t) {
                const int k = std::min(std::max(dir ? nz - 1 - t : t, 0), nz - 1);
                mgk::StepCoef<T>& q = tab[(size_t(dir) * nJ + J) * mgk::kStepStride + t];
                q.tl = T(s.Tlam[size_t(k) * nJ + J]);
                q.ts = T(s.Tth[size_t(k) * (nJ + 1) + J]);
                q.tn = T(s.Tth[size_t(k) * (nJ + 1) + J + 1]);
                q.tc = T(s.Tr[size_t(dir ? k : k + 1) * nJ + J]);
            }
    return tab;
}

template <typename T, typename S>
mg_status upload(mg_handle* h, T** dst, const std::vector<S>& src) {
    MG_TRY(dalloc(h, dst, src.size()));
    std::vector<T> tmp(src.begin(), src.end());
    if (!tmp.empty())
        HIP_TRY(h, hipMemcpyAsync(*dst, tmp.data(), tmp.size() * sizeof(T),
                                  hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MG_OK;
}

template <typename T>
mgk::LevelView<T> view(const DevLevel& d);

template <>
mgk::LevelView<float> view<float>(const DevLevel& d) {
    return {d.nI, d.nJ, d.nz, d.plane, d.Tlam32, d.Tth32, d.Tr32, d.M32, d.invp32, d.sc32};
}
template <>
mgk::LevelView<double> view<double>(const DevLevel& d) {
    return {d.nI, d.nJ, d.nz, d.plane, d.Tlam64, d.Tth64, d.Tr64, d.M64, d.invp64, d.sc64};
}

template <typename T>
mgk::TransferView<T> xview(const DevLevel& f, const DevLevel& c);
template <>
mgk::TransferView<float> xview<float>(const DevLevel& f, const DevLevel& c) {
    return {c.nI, c.nJ, f.crow_of, f.prow, f.pw32, c.child_first, c.child_count, c.ptrow,
            c.ptw32};
}
template <>
mgk::TransferView<double> xview<double>(const DevLevel& f, const DevLevel& c) {
    return {c.nI, c.nJ, f.crow_of, f.prow, f.pw64, c.child_first, c.child_count, c.ptrow,
            c.ptw64};
}

template <typename T>
Work<T>& work(DevLevel& d);
template <>
Work<float>& work<float>(DevLevel& d) { return d.w32; }
template <>
Work<double>& work<double>(DevLevel& d) { return d.w64; }

template <typename T>
const T* dense_C(const mg_handle* h, bool transposed);
template <>
const float* dense_C<float>(const mg_handle* h, bool transposed) {
    return transposed ? h->dense.Ct32 : h->dense.C32;
}
template <>
const double* dense_C<double>(const mg_handle* h, bool transposed) {
    return transposed ? h->dense.Ct64 : h->dense.C64;
}

template <typename T>
mg_status ensure_work(mg_handle* h) {
    bool& have = std::is_same<T, float>::value ? h->have32 : h->have64;
    if (have) return MG_OK;
    for (auto& d : h->lv) {
        Work<T>& w = work<T>(d);
        for (T** p : {&w.f, &w.xa, &w.xb})
            MG_TRY(dalloc(h, p, d.n));
    }
    have = true;
    return MG_OK;
}

// --- profiling ----------------------------------------------------------------
hipEvent_t next_event(mg_handle* h) {
    if (h->no_events) return nullptr;
    if (h->next_event == h->events.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->events.push_back(e);
    }
    return h->events[h->next_event++];
}

struct Launch {
    mg_handle* h;
    ProfRec rec{};
    bool on = false;
    Launch(mg_handle* hh, int cls, int level, double bytes) : h(hh) {
        h->alg_bytes += bytes;
        // profile 1: finest level only (no events around the short coarse
        // launches); 2: every launch; 3: none (see SweepGroup)
        if (!h->opt.profile || h->opt.profile == 3 || (h->opt.profile == 1 && level != 0))
            return;
        rec.cls = cls;
        rec.level = level;
        rec.bytes = bytes;
        rec.a = next_event(h);
        rec.b = next_event(h);
        if (rec.a && rec.b) {
            on = true;
            (void)hipEventRecord(rec.a, h->stream);
        }
    }
    ~Launch() {
        if (!on) return;
        (void)hipEventRecord(rec.b, h->stream);
        h->recs.push_back(rec);
    }
};

// Profile 3: one pair of events around the consecutive post-smoothing
// sweeps of the finest level in each forward V-cycle, recorded as that many
// launches of the sweep. Every event pair between two kernels leaves the GPU
// idle for a few microseconds; two per cycle time the dominant kernel at a
// quarter of the cost of a pair around each of its launches.
struct SweepGroup {
    mg_handle* h;
    ProfRec rec{};
    bool on = false;
    SweepGroup(mg_handle* hh, int level, int launches, double bytes) : h(hh) {
        if (h->opt.profile != 3 || level != 0 || launches <= 0) return;
        rec.cls = MG_K_SMOOTH;
        rec.level = level;
        rec.bytes = bytes;
        rec.launches = launches;
        rec.a = next_event(h);
        rec.b = next_event(h);
        if (rec.a && rec.b) {
            on = true;
            (void)hipEventRecord(rec.a, h->stream);
        }
    }
    ~SweepGroup() {
        if (!on) return;
        (void)hipEventRecord(rec.b, h->stream);
        h->recs.push_back(rec);
    }
};

void prof_reset(mg_handle* h) {
    h->recs.clear();
    h->phases.clear();
    h->next_event = 0;
    h->alg_bytes = 0;
}

// Events around one phase of the outer loop (a V-cycle or a refinement
// step), summed into mg_stats.ms_vcycle / ms_residual; with profile 1 and 2
// only (an event pair between two kernels idles the GPU for microseconds).
struct Phase {
    mg_handle* h;
    ProfRec rec{};
    bool on = false;
    Phase(mg_handle* hh, int kind) : h(hh) {
        if (h->opt.profile != 1 && h->opt.profile != 2) return;
        rec.cls = kind;
        rec.a = next_event(h);
        rec.b = next_event(h);
        if (rec.a && rec.b) {
            on = true;
            (void)hipEventRecord(rec.a, h->stream);
        }
    }
    ~Phase() {
        if (!on) return;
        (void)hipEventRecord(rec.b, h->stream);
        h->phases.push_back(rec);
    }
};

void prof_collect(mg_handle* h, mg_stats* st) {
    if (!st) return;
    st->ms_vcycle = st->ms_residual = 0;
    for (const ProfRec& r : h->phases) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
        (r.cls == 0 ? st->ms_vcycle : st->ms_residual) += ms;
    }
    for (int c = 0; c < MG_NK; ++c) {
        st->kern_ms[c] = st->kern_bytes[c] = st->kern_fine_ms[c] = st->kern_fine_bytes[c] = 0;
        st->kern_launches[c] = st->kern_fine_launches[c] = 0;
    }
    for (const ProfRec& r : h->recs) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
        st->kern_ms[r.cls] += ms;
        st->kern_bytes[r.cls] += r.bytes;
        st->kern_launches[r.cls] += r.launches;
        if (r.level == 0) {
            st->kern_fine_ms[r.cls] += ms;
            st->kern_fine_bytes[r.cls] += r.bytes;
            st->kern_fine_launches[r.cls] += r.launches;
        }
    }
}

mg_status check_launch(mg_handle* h, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(h, MG_ERR_HIP, "launch of %s failed: %s", what,
                                     hipGetErrorString(e));
    return MG_OK;
}

// --- level operations with byte accounting ---------------------------------------
template <typename T>
mg_status op_smooth(mg_handle* h, int l, const T* f, const T* xin, T* xout, int cls,
                    double omega) {
    DevLevel& d = h->lv[l];
    // a Jacobi sweep reads the old iterate of the neighbour columns while
    // others are written: it must never run in place
    if (xin == xout || f == xout)
        return fail(h, MG_ERR_ARG, "internal: sweep on level %d would overwrite its input", l);
    const double bytes = double(d.n) * sizeof(T) * (xin ? 4 : 3);
    {
        Launch g(h, cls, l, bytes);
        mgk::smooth<T>(view<T>(d), f, xin, xout, T(omega), h->opt.staged_columns, h->stream);
    }
    return check_launch(h, "smooth");
}

template <typename T>
mg_status op_restrict(mg_handle* h, int l, const T* f, const T* x, T* fc) {
    DevLevel &d = h->lv[l], &c = h->lv[l + 1];
    const double bytes = double(d.n) * sizeof(T) * (x ? 3 : 1) + double(c.n) * sizeof(T);
    {
        Launch g(h, MG_K_RESTRICT, l, bytes);
        mgk::restrict_residual<T>(view<T>(d), xview<T>(d, c), f, x, fc, h->stream);
    }
    return check_launch(h, "restrict_residual");
}

template <typename T>
mg_status op_prolong(mg_handle* h, int l, const T* xc, T* x) {
    DevLevel &d = h->lv[l], &c = h->lv[l + 1];
    const double bytes = double(d.n) * sizeof(T) * 2 + double(c.n) * sizeof(T);
    {
        Launch g(h, MG_K_PROLONG, l, bytes);
        mgk::prolong_add<T>(view<T>(d), xview<T>(d, c), xc, x, h->stream);
    }
    return check_launch(h, "prolong_add");
}

template <typename T>
mg_handle::CoarseGraph& coarse_graph(mg_handle* h) {
    return std::is_same<T, float>::value ? h->g32 : h->g64;
}

// One V-cycle from zero on level l; returns the buffer holding the result.
template <typename T>
mg_status vcycle(mg_handle* h, int l, const T* f, T** result) {
    DevLevel& d = h->lv[l];
    Work<T>& w = work<T>(d);
    const int last = int(h->lv.size()) - 1;
    if (l == 1 && !h->capturing && !h->no_graphs && h->opt.profile != 2) {
        mg_handle::CoarseGraph& G = coarse_graph<T>(h);
        if (G.exec && G.dense_valid == h->dense.valid && f == w.f) {
            HIP_TRY(h, hipGraphLaunch(G.exec, h->stream));
            h->alg_bytes += G.bytes;
            *result = static_cast<T*>(G.result);
            return MG_OK;
        }
    }
    T* cur = w.xa;
    T* nxt = w.xb;
    if (l == last) {
        if (h->dense.valid) {
            // the coarse solve's explicit matrix: one matrix-vector product
            {
                Launch g(h, MG_K_COARSE, l, double(d.n) * (d.n + 2) * sizeof(T));
                mgk::dense_matvec<T>(dense_C<T>(h, false), d.n, f, cur, h->stream);
            }
            MG_TRY(check_launch(h, "dense coarse solve"));
            *result = cur;
            return MG_OK;
        }
        if (d.plane <= mgk::kCoarseSolveColumns) {
            // all coarse sweeps in one single-block launch
            int where = 0;
            {
                Launch g(h, MG_K_COARSE, l,
                         double(d.n) * sizeof(T) * (3.0 + 4.0 * (h->opt.coarse_sweeps - 1)));
                where = mgk::coarse_solve<T>(view<T>(d), f, cur, nxt, T(h->opt.omega),
                                             h->opt.coarse_sweeps, h->max_lds, h->stream);
            }
            MG_TRY(check_launch(h, "coarse_solve"));
            *result = where == 0 ? cur : nxt;
            return MG_OK;
        }
        MG_TRY(op_smooth<T>(h, l, f, nullptr, cur, MG_K_COARSE, h->opt.omega));
        for (int s = 1; s < h->opt.coarse_sweeps; ++s) {
            MG_TRY(op_smooth<T>(h, l, f, cur, nxt, MG_K_COARSE, h->opt.omega));
            std::swap(cur, nxt);
        }
        *result = cur;
        return MG_OK;
    }
    const int nu1 = h->opt.nu_pre, nu2 = h->opt.nu_post;
    MG_TRY(op_smooth<T>(h, l, f, nullptr, cur, MG_K_SMOOTH0, mgs::sweep_omega(h->opt, nu1, 0)));
    for (int s = 1; s < nu1; ++s) {
        MG_TRY(op_smooth<T>(h, l, f, cur, nxt, MG_K_SMOOTH, mgs::sweep_omega(h->opt, nu1, s)));
        std::swap(cur, nxt);
    }
    Work<T>& wc = work<T>(h->lv[l + 1]);
    MG_TRY(op_restrict<T>(h, l, f, cur, wc.f));
    T* xc = nullptr;
    MG_TRY(vcycle<T>(h, l + 1, wc.f, &xc));
    MG_TRY(op_prolong<T>(h, l, xc, cur));
    {
        SweepGroup g(h, l, nu2, double(nu2) * double(d.n) * sizeof(T) * 4);
        for (int s = 0; s < nu2; ++s) {
            MG_TRY(op_smooth<T>(h, l, f, cur, nxt, MG_K_SMOOTH,
                                mgs::sweep_omega(h->opt, nu2, s)));
            std::swap(cur, nxt);
        }
    }
    *result = cur;
    return MG_OK;
}

// Capture the V-cycle of levels 1..L-1 in precision T as a graph (on the
// handle's private stream; nothing in it is a memset or an event), for the
// current options, work buffers and coarsest-level route. Graphs are an
// optimisation: a capture that fails leaves the cycle to direct launches.
template <typename T>
mg_status capture_coarse(mg_handle* h) {
    mg_handle::CoarseGraph& G = coarse_graph<T>(h);
    if (G.exec) {
        (void)hipGraphExecDestroy(G.exec);
        G.exec = nullptr;
    }
    const bool have = std::is_same<T, float>::value ? h->have32 : h->have64;
    if (h->lv.size() < 2 || !have || !h->cap_stream || !h->opt.graphs) return MG_OK;
    hipStream_t user = h->stream;
    const int profile = h->opt.profile;
    const double bytes0 = h->alg_bytes;
    h->stream = h->cap_stream;
    h->opt.profile = 0;
    h->no_events = true;
    h->capturing = true;
    T* res = nullptr;
    hipGraph_t graph = nullptr;
    mg_status s = MG_OK;
    if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        s = vcycle<T>(h, 1, work<T>(h->lv[1]).f, &res);
        if (hipStreamEndCapture(h->cap_stream, &graph) != hipSuccess) graph = nullptr;
    }
    (void)hipGetLastError();
    h->stream = user;
    h->opt.profile = profile;
    h->no_events = false;
    h->capturing = false;
    G.bytes = h->alg_bytes - bytes0;
    h->alg_bytes = bytes0;
    if (s == MG_OK && graph &&
        hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0) == hipSuccess) {
        G.result = res;
        G.dense_valid = h->dense.valid;
    } else {
        G.exec = nullptr;
        (void)hipGetLastError();
    }
    if (graph) (void)hipGraphDestroy(graph);
    return MG_OK;
}

mg_status capture_graphs(mg_handle* h) {
    MG_TRY(capture_coarse<float>(h));
    return capture_coarse<double>(h);
}

template <typename T>
mg_status op_restrict_T(mg_handle* h, int l, const T* f, const T* x, T* r, T* fc) {
    DevLevel &d = h->lv[l], &c = h->lv[l + 1];
    {
        Launch g(h, MG_K_RESTRICT, l, double(d.n) * sizeof(T) * 4);
        mgk::apply<T>(view<T>(d), x, f, r, h->stream);
    }
    MG_TRY(check_launch(h, "apply"));
    {
        Launch g(h, MG_K_RESTRICT, l, double(d.n) * sizeof(T) + double(c.n) * sizeof(T));
        mgk::prolong_transpose<T>(view<T>(d), xview<T>(d, c), r, fc, h->stream);
    }
    return check_launch(h, "prolong_transpose");
}

template <typename T>
mg_status op_inject(mg_handle* h, int l, const T* xc, T* x) {
    DevLevel &d = h->lv[l], &c = h->lv[l + 1];
    {
        Launch g(h, MG_K_PROLONG, l, double(d.n) * sizeof(T) * 2 + double(c.n) * sizeof(T));
        mgk::inject_add<T>(view<T>(d), xview<T>(d, c), xc, x, h->stream);
    }
    return check_launch(h, "inject_add");
}

// The transposed V-cycle from zero on level l (the transpose of the map
// f -> vcycle(f)); returns the buffer holding the result. A transposed sweep
// sends (xbar, fbar) to (xbar - omega H H_z^{-1} xbar, fbar + omega H_z^{-1}
// xbar): the step of a sweep on the right-hand side xbar whose iterate is
// fbar and whose residual is xbar. So the transposed steps, taken in reverse
// order, are forward sweeps from zero (factors reversed), the transposes of
// the transfers (P^T restricts the residual, R^T injects the correction) and
// the transposed coarse solve.
template <typename T>
mg_status vcycle_adj(mg_handle* h, int l, const T* f, T** result) {
    DevLevel& d = h->lv[l];
    Work<T>& w = work<T>(d);
    const int last = int(h->lv.size()) - 1;
    T* cur = w.xa;
    T* nxt = w.xb;
    if (l == last) {
        if (h->dense.valid) {
            {
                Launch g(h, MG_K_COARSE, l, double(d.n) * (d.n + 2) * sizeof(T));
                mgk::dense_matvec<T>(dense_C<T>(h, true), d.n, f, cur, h->stream);
            }
            MG_TRY(check_launch(h, "dense transposed coarse solve"));
            *result = cur;
            return MG_OK;
        }
        // sweeps from zero with one factor: a symmetric map, its own transpose
        return vcycle<T>(h, l, f, result);
    }
    const int nu1 = h->opt.nu_pre, nu2 = h->opt.nu_post;
    Work<T>& wc = work<T>(h->lv[l + 1]);
    if (nu2 > 0) {
        MG_TRY(op_smooth<T>(h, l, f, nullptr, cur, MG_K_SMOOTH0,
                            mgs::sweep_omega(h->opt, nu2, nu2 - 1)));
        for (int s = nu2 - 2; s >= 0; --s) {
            MG_TRY(op_smooth<T>(h, l, f, cur, nxt, MG_K_SMOOTH, mgs::sweep_omega(h->opt, nu2, s)));
            std::swap(cur, nxt);
        }
        MG_TRY(op_restrict_T<T>(h, l, f, cur, nxt, wc.f));
    } else {
        // no sweeps: the iterate is zero and its residual is f
        {
            DevLevel& c = h->lv[l + 1];
            Launch g(h, MG_K_RESTRICT, l, double(d.n) * sizeof(T) + double(c.n) * sizeof(T));
            mgk::prolong_transpose<T>(view<T>(d), xview<T>(d, c), f, wc.f, h->stream);
        }
        MG_TRY(check_launch(h, "prolong_transpose"));
        mgk::fill<T>(cur, T(0), d.n, h->stream);
        MG_TRY(check_launch(h, "fill"));
    }
    T* xc = nullptr;
    MG_TRY(vcycle_adj<T>(h, l + 1, wc.f, &xc));
    MG_TRY(op_inject<T>(h, l, xc, cur));
    {
        SweepGroup g(h, l, nu1, double(nu1) * double(d.n) * sizeof(T) * 4);
        for (int s = nu1 - 1; s >= 0; --s) {
            MG_TRY(op_smooth<T>(h, l, f, cur, nxt, MG_K_SMOOTH, mgs::sweep_omega(h->opt, nu1, s)));
            std::swap(cur, nxt);
        }
    }
    *result = cur;
    return MG_OK;
}

// Copy the reduced scalar to the host (asynchronously; the copy's completion
// is the event scalar_ready), and wait for it. Waiting on the event, not the
// stream, lets work enqueued after the copy keep the GPU busy meanwhile.
mg_status post_scalar(mg_handle* h) {
    HIP_TRY(h, hipMemcpyAsync(h->host_scalar, h->scalar, 2 * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipEventRecord(h->scalar_ready, h->stream));
    return MG_OK;
}

mg_status wait_scalar(mg_handle* h, double* out) {
    HIP_TRY(h, hipEventSynchronize(h->scalar_ready));
    *out = *h->host_scalar;
    return MG_OK;
}

mg_status sync_scalar(mg_handle* h, double* out) {
    MG_TRY(post_scalar(h));
    return wait_scalar(h, out);
}

// FP64 update + residual step; returns ||r||.
// One refinement step with the iterate, b and H in precision U (FP64, or
// FP32 in the pure single-precision solve) and the correction e and
// residual r in the V-cycle's precision T.
// Enqueues the step; its ||r||^2 (and ||b||^2 with with_bnorm, summed in the
// same pass) reaches the host with post_scalar, read by finish_step.
template <typename T, typename U>
mg_status refine_step(mg_handle* h, const U* b, const U* uin, const T* e, U* uout, T* r,
                      bool with_bnorm = false) {
    DevLevel& d = h->lv[0];
    // b read, r written; u and the mass read unless u is zero and stays
    // so; e read and the new u written when there is an update
    const double bytes =
        double(d.n) * (sizeof(U) + sizeof(T) + (uin ? sizeof(U) : 0) +
                       (uin || e ? sizeof(U) : 0) + (e ? sizeof(T) + sizeof(U) : 0));
    int nb = 0;
    {
        Phase ph(h, 1);
        {
            Launch g(h, MG_K_RESIDUAL64, 0, bytes);
            nb = mgk::residual_update<U, T, T>(view<U>(d), b, uin, e, uout, r, h->partials,
                                               with_bnorm ? h->partials + h->max_partials
                                                          : nullptr,
                                               h->stream);
        }
        MG_TRY(check_launch(h, "residual_update"));
        {
            Launch g(h, MG_K_OTHER, 0, double(nb) * 8 * (with_bnorm ? 2 : 1));
            mgk::sum_partials(h->partials, nb, h->scalar, h->stream, with_bnorm ? 2 : 1,
                              h->max_partials);
        }
    }
    return post_scalar(h);
}

// ||r|| of the last step (and ||b|| into bnorm when given, for a step
// enqueued with with_bnorm).
mg_status finish_step(mg_handle* h, double* rnorm, double* bnorm = nullptr) {
    double s2 = 0;
    MG_TRY(wait_scalar(h, &s2));
    *rnorm = std::sqrt(s2);
    if (bnorm) *bnorm = std::sqrt(h->host_scalar[1]);
    return MG_OK;
}

// The outer refinement loop: V-cycles in precision T, the iterate and its
// residual in precision U (FP64; FP32 for MG_PREC_FP32, where b and u are
// cast on entry and u back on exit), with the forward (transposed = false)
// or transposed V-cycle.
// zero: start from u = 0 whatever u holds (u is then written only).
template <typename T, typename U>
mg_status outer(mg_handle* h, const double* b, double* u, double tol, mg_stats* st,
                bool transposed, bool zero, bool* stalled = nullptr) {
    if (!(std::is_same<T, float>::value ? h->have32 : h->have64)) {
        // first use of this precision (the FP64 fallback of a mixed solve)
        MG_TRY(ensure_work<T>(h));
        MG_TRY(capture_coarse<T>(h));
    }
    DevLevel& d = h->lv[0];
    Work<T>& w = work<T>(d);
    auto t0 = std::chrono::steady_clock::now();
    prof_reset(h);
    double bnorm = 0;
    const U* bU = nullptr;
    U *ucur = nullptr, *unext = nullptr;
    // ucur == nullptr: the iterate is zero (a solve from u = 0 before its
    // first update)
    if constexpr (std::is_same<U, double>::value) {
        bU = b;
        ucur = zero ? nullptr : u;
    } else {
        if (!h->b32) {
            MG_TRY(dalloc(h, &h->b32, d.n));
            MG_TRY(dalloc(h, &h->u32a, d.n));
            MG_TRY(dalloc(h, &h->u32b, d.n));
        }
        {
            Launch g(h, MG_K_OTHER, 0, double(d.n) * (zero ? 12 : 24));
            mgk::cast<double, float>(b, h->b32, d.n, h->stream);
            if (!zero) mgk::cast<double, float>(u, h->u32a, d.n, h->stream);
        }
        MG_TRY(check_launch(h, "cast"));
        bU = h->b32;
        ucur = zero ? nullptr : h->u32a;
    }
    // r0 = b - H u0 (the fine-level right-hand side of the first V-cycle)
    T* r = w.f;
    double rn = 0;
    // (||b|| in the same pass)
    MG_TRY((refine_step<T, U>(h, bU, ucur, nullptr, nullptr, r, true)));
    // enqueue one V-cycle on r; its correction e is what the next step adds
    auto cycle = [&](const T** e) -> mg_status {
        Phase ph(h, 0);
        T* x = nullptr;
        if (!transposed) MG_TRY(vcycle<T>(h, 0, w.f, &x));
        else MG_TRY(vcycle_adj<T>(h, 0, w.f, &x));
        *e = x;
        return MG_OK;
    };
    // The first cycle is almost always needed: enqueue it before the wait
    // (wasted only when u0 already meets the tolerance).
    const T* e_ahead = nullptr;   // a V-cycle already enqueued on the current r
    if (h->opt.max_iters > 0) MG_TRY(cycle(&e_ahead));
    MG_TRY(finish_step(h, &rn, &bnorm));
    // residual norms, kept in place (no allocation inside a solve)
    struct Hist {
        double v[MG_HIST];
        size_t n = 0;
        void push_back(double x) { v[n < MG_HIST ? n++ : MG_HIST - 1] = x; }
        size_t size() const { return n; }
        double back() const { return v[n - 1]; }
        double operator[](size_t i) const { return v[i]; }
    } hist;
    hist.push_back(rn);
    int it = 0, slow = 0;
    mg_status status = MG_OK;
    if (!std::isfinite(rn) || !std::isfinite(bnorm)) status = MG_ERR_BREAKDOWN;
    while (status == MG_OK) {
        if (rn <= tol * bnorm) break;
        if (it >= h->opt.max_iters) {
            status = MG_ERR_NOT_CONVERGED;
            break;
        }
        const T* e = e_ahead;
        if (!e) MG_TRY(cycle(&e));
        e_ahead = nullptr;
        // the last contraction factor, carried forward to predict ||r||
        const double rho = hist.size() >= 2 ? hist.back() / hist[hist.size() - 2] : 1.0;
        if constexpr (std::is_same<U, double>::value) {
            // The step predicted to be the last writes into the caller's u
            // (when it does not read it), the others alternate between two
            // buffers of their own: no copy at the end unless the prediction
            // misses.
            if (rn * std::min(rho, 1.0) <= tol * bnorm && ucur != u) unext = u;
            else unext = ucur == h->u_alt ? h->u_alt2 : h->u_alt;
        } else {
            unext = ucur == h->u32a ? h->u32b : h->u32a;
        }
        MG_TRY((refine_step<T, U>(h, bU, ucur, e, unext, r)));
        // While the new norm travels to the host, keep the GPU busy with the
        // next V-cycle when the residual is predicted to stay well above the
        // tolerance. The update itself waits for the norm, so a cycle
        // enqueued in vain costs time only, never the result.
        if (it + 1 < h->opt.max_iters && std::isfinite(rho) &&
            rn * std::min(rho, 1.0) > 3.0 * tol * bnorm)
            MG_TRY(cycle(&e_ahead));
        MG_TRY(finish_step(h, &rn));
        std::swap(ucur, unext);
        ++it;
        hist.push_back(rn);
        if (h->log)
            std::fprintf(stderr, "mg: %s%s iteration %d relres %.3e factor %.3f\n",
                         std::is_same<T, float>::value ? "fp32 cycle" : "fp64 cycle",
                         transposed ? " (adjoint)" : "", it, bnorm > 0 ? rn / bnorm : 0.0,
                         hist[hist.size() - 2] > 0 ? rn / hist[hist.size() - 2] : 0.0);
        if (!std::isfinite(rn)) status = MG_ERR_BREAKDOWN;
        // stagnation guard: the caller continues with FP64 cycles
        if (stalled && h->opt.stall_iters > 0 && status == MG_OK) {
            slow = rn > h->opt.stall_factor * hist[hist.size() - 2] ? slow + 1 : 0;
            if (slow >= h->opt.stall_iters && rn > tol * bnorm) {
                *stalled = true;
                break;
            }
        }
    }
    if (!ucur) {
        // no update was made from u = 0 (b meets the tolerance, or max_iters
        // is 0): the solution is zero (a fill kernel, not a memset)
        {
            Launch g(h, MG_K_OTHER, 0, double(d.n) * 8);
            mgk::fill<double>(u, 0.0, d.n, h->stream);
        }
        MG_TRY(check_launch(h, "fill"));
    } else if constexpr (std::is_same<U, double>::value) {
        if (ucur != u) {
            Launch g(h, MG_K_OTHER, 0, double(d.n) * 16);
            HIP_TRY(h, hipMemcpyAsync(u, ucur, d.n * sizeof(double), hipMemcpyDeviceToDevice,
                                      h->stream));
        }
    } else {
        {
            Launch g(h, MG_K_OTHER, 0, double(d.n) * 12);
            mgk::cast<float, double>(ucur, u, d.n, h->stream);
        }
        MG_TRY(check_launch(h, "cast"));
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    auto t1 = std::chrono::steady_clock::now();
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->iters = it;
        st->relres = bnorm > 0 ? rn / bnorm : 0.0;
        for (size_t m = 0; m < hist.size() && m < MG_HIST; ++m) st->res_hist[m] = hist[m];
        st->ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
        st->levels_used = int(h->lv.size());
        st->alg_bytes = h->alg_bytes;
        prof_collect(h, st);
    }
    if (status == MG_ERR_BREAKDOWN)
        return fail(h, status, "non-finite residual norm at iteration %d", it);
    if (status == MG_ERR_NOT_CONVERGED)
        h->err = "max_iters reached before the tolerance";
    return status;
}

// Form the coarsest solve's matrices for the current pivots, omega and
// number of sweeps: C^T from the solves of the unit vectors (FP64), C by
// transposition, FP32 copies of both.
mg_status rebuild_dense(mg_handle* h) {
    DenseCoarse& D = h->dense;
    D.valid = false;
    if (!D.enabled) return MG_OK;
    const DevLevel& c = h->lv.back();
    if (!mgk::coarse_basis(view<double>(c), D.Ct64, h->opt.omega, h->opt.coarse_sweeps,
                           h->max_lds, h->stream)) {
        D.enabled = false;   // does not fit: keep the sweeps
        return MG_OK;
    }
    MG_TRY(check_launch(h, "coarse_basis"));
    mgk::transpose_square<double>(D.Ct64, D.C64, D.n, h->stream);
    MG_TRY(check_launch(h, "transpose"));
    mgk::cast<double, float>(D.C64, D.C32, D.n * D.n, h->stream);
    mgk::cast<double, float>(D.Ct64, D.Ct32, D.n * D.n, h->stream);
    MG_TRY(check_launch(h, "cast"));
    D.sweeps = h->opt.coarse_sweeps;
    D.omega = h->opt.omega;
    D.valid = true;
    return MG_OK;
}

// Device-side coefficients: masses per level, pivots, FP32 copies.
mg_status set_coeffs(mg_handle* h, const double* alpha) {
    DevLevel& f = h->lv[0];
    // count the bad values before anything is written: a rejected alpha
    // leaves the handle's operator as it was
    int nb = mgk::fine_mass(view<double>(f), f.V64, alpha, nullptr, h->partials, h->stream);
    mgk::sum_partials(h->partials, nb, h->scalar, h->stream);
    MG_TRY(check_launch(h, "alpha check"));
    double bad = 0;
    MG_TRY(sync_scalar(h, &bad));
    if (bad != 0)
        return fail(h, MG_ERR_ARG, "alpha has %.0f values that are not finite and > 0", bad);
    mgk::fine_mass(view<double>(f), f.V64, alpha, f.M64, h->partials, h->stream);
    MG_TRY(check_launch(h, "fine_mass"));
    for (size_t l = 0; l + 1 < h->lv.size(); ++l) {
        DevLevel &d = h->lv[l], &c = h->lv[l + 1];
        mgk::restrict_residual<double>(view<double>(d), xview<double>(d, c), d.M64, nullptr,
                                       c.M64, h->stream);
        MG_TRY(check_launch(h, "mass aggregation"));
    }
    for (auto& d : h->lv) {
        mgk::pivots(view<double>(d), d.invp64, d.invp32, d.M32, h->stream);
        MG_TRY(check_launch(h, "pivots"));
    }
    MG_TRY(rebuild_dense(h));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return MG_OK;
}

mg_status build(mg_handle* h, const double* alpha) {
    std::string e = mgs::plan(h->grid, h->opt.levels, h->opt.semi_threshold, h->host);
    if (!e.empty()) return fail(h, MG_ERR_ARG, "%s", e.c_str());
    const size_t L = h->host.levels.size();
    h->lv.resize(L);
    for (size_t l = 0; l < L; ++l) {
        const mgs::Level& s = h->host.levels[l];
        DevLevel& d = h->lv[l];
        d.nI = s.nI;
        d.nJ = s.nJ;
        d.nz = s.nz;
        d.plane = (long long)s.nI * s.nJ;
        d.n = d.plane * s.nz;
        MG_TRY(upload(h, &d.Tlam64, s.Tlam));
        MG_TRY(upload(h, &d.Tth64, s.Tth));
        MG_TRY(upload(h, &d.Tr64, s.Tr));
        MG_TRY(upload(h, &d.V64, s.V));
        MG_TRY(upload(h, &d.Tlam32, s.Tlam));
        MG_TRY(upload(h, &d.Tth32, s.Tth));
        MG_TRY(upload(h, &d.Tr32, s.Tr));
        MG_TRY(upload(h, &d.sc64, step_table<double>(s)));
        MG_TRY(upload(h, &d.sc32, step_table<float>(s)));
        MG_TRY(dalloc(h, &d.M64, d.n));
        MG_TRY(dalloc(h, &d.invp64, d.n));
        MG_TRY(dalloc(h, &d.M32, d.n));
        MG_TRY(dalloc(h, &d.invp32, d.n));
        if (l + 1 < L) {
            MG_TRY(upload(h, &d.crow_of, s.crow_of));
            MG_TRY(upload(h, &d.prow, s.prow));
            MG_TRY(upload(h, &d.pw64, s.pw));
            MG_TRY(upload(h, &d.pw32, s.pw));
        }
        if (l > 0) {
            MG_TRY(upload(h, &d.child_first, s.child_first));
            MG_TRY(upload(h, &d.child_count, s.child_count));
            MG_TRY(upload(h, &d.ptrow, s.ptrow));
            MG_TRY(upload(h, &d.ptw64, s.ptw));
            MG_TRY(upload(h, &d.ptw32, s.ptw));
        }
    }
    DevLevel& f = h->lv[0];
    h->max_partials = std::max({mgk::residual_update_blocks(view<double>(f)),
                                mgk::blocks_for(f.plane), 8192});
    MG_TRY(dalloc(h, &h->partials, 2 * size_t(h->max_partials)));
    MG_TRY(dalloc(h, &h->scalar, 2));
    MG_TRY(dalloc(h, &h->u_alt, f.n));
    MG_TRY(dalloc(h, &h->u_alt2, f.n));
    HIP_TRY(h, hipHostMalloc((void**)&h->host_scalar, 2 * sizeof(double), hipHostMallocDefault));
    HIP_TRY(h, hipEventCreateWithFlags(&h->scalar_ready, hipEventDisableTiming));
    {
        int dev = 0, lds = 0;
        HIP_TRY(h, hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                hipSuccess && lds > 0)
            h->max_lds = size_t(lds);
        (void)hipGetLastError();
    }
    {
        const DevLevel& c = h->lv.back();
        DenseCoarse& D = h->dense;
        D.n = c.n;
        D.enabled = c.n <= mgk::kDenseCoarseMax && c.plane <= mgk::kCoarseLdsColumns &&
                    mgk::coarse_lds_bytes<double>(c.plane, c.nJ, c.nz, true) <= h->max_lds;
        if (D.enabled) {
            const size_t nn = size_t(c.n) * size_t(c.n);
            MG_TRY(dalloc(h, &D.C64, nn));
            MG_TRY(dalloc(h, &D.Ct64, nn));
            MG_TRY(dalloc(h, &D.C32, nn));
            MG_TRY(dalloc(h, &D.Ct32, nn));
        }
    }
    return set_coeffs(h, alpha);
}

void release(mg_handle* h) {
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (mg_handle::CoarseGraph* G : {&h->g32, &h->g64})
        if (G->exec) (void)hipGraphExecDestroy(G->exec);
    h->g32.exec = h->g64.exec = nullptr;
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    h->cap_stream = nullptr;
    for (void* p : h->allocs) (void)hipFree(p);
    h->allocs.clear();
    if (h->host_scalar) (void)hipHostFree(h->host_scalar);
    h->host_scalar = nullptr;
    if (h->scalar_ready) (void)hipEventDestroy(h->scalar_ready);
    h->scalar_ready = nullptr;
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    h->events.clear();
}

bool shape_ok(const mg_handle* h, int l) { return h && l >= 0 && l < int(h->lv.size()); }

// Cast an FP64 field into a level buffer of precision T (copy for FP64).
template <typename T>
void to_level(mg_handle* h, const double* src, T* dst, long long n) {
    mgk::cast<double, T>(src, dst, n, h->stream);
}
template <typename T>
void from_level(mg_handle* h, const T* src, double* dst, long long n) {
    mgk::cast<T, double>(src, dst, n, h->stream);
}

template <typename T>
mg_status level_sweep(mg_handle* h, int l, const double* f, const double* xin, double* xout) {
    MG_TRY(ensure_work<T>(h));
    DevLevel& d = h->lv[l];
    Work<T>& w = work<T>(d);
    to_level<T>(h, f, w.f, d.n);
    if (xin) to_level<T>(h, xin, w.xa, d.n);
    MG_TRY(op_smooth<T>(h, l, w.f, xin ? w.xa : nullptr, w.xb,
                        xin ? MG_K_SMOOTH : MG_K_SMOOTH0, h->opt.omega));
    from_level<T>(h, w.xb, xout, d.n);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_launch(h, "level_sweep");
}

template <typename T>
mg_status level_restrict(mg_handle* h, int l, const double* f, const double* x, double* fc) {
    MG_TRY(ensure_work<T>(h));
    DevLevel &d = h->lv[l], &c = h->lv[l + 1];
    Work<T>& w = work<T>(d);
    Work<T>& wc = work<T>(c);
    to_level<T>(h, f, w.f, d.n);
    if (x) to_level<T>(h, x, w.xa, d.n);
    MG_TRY(op_restrict<T>(h, l, w.f, x ? w.xa : nullptr, wc.f));
    from_level<T>(h, wc.f, fc, c.n);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_launch(h, "level_residual_restrict");
}

template <typename T>
mg_status level_prolong(mg_handle* h, int l, const double* xc, double* x) {
    MG_TRY(ensure_work<T>(h));
    DevLevel &d = h->lv[l], &c = h->lv[l + 1];
    Work<T>& w = work<T>(d);
    Work<T>& wc = work<T>(c);
    to_level<T>(h, xc, wc.xa, c.n);
    to_level<T>(h, x, w.xa, d.n);
    MG_TRY(op_prolong<T>(h, l, wc.xa, w.xa));
    from_level<T>(h, w.xa, x, d.n);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_launch(h, "level_prolong_add");
}

template <typename T>
mg_status one_vcycle(mg_handle* h, const double* f, double* x, bool transposed) {
    MG_TRY(ensure_work<T>(h));
    DevLevel& d = h->lv[0];
    Work<T>& w = work<T>(d);
    to_level<T>(h, f, w.f, d.n);
    T* out = nullptr;
    if (!transposed) MG_TRY(vcycle<T>(h, 0, w.f, &out));
    else MG_TRY(vcycle_adj<T>(h, 0, w.f, &out));
    from_level<T>(h, out, x, d.n);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_launch(h, "vcycle");
}

// Scratch of mg_solve_noalloc: the per-block norm partials of the
// refinement steps and the two reduced norms, in a device array of the
// library's own. Each GPU holds one copy (until the process ends); its
// address there is looked up once, at the first mg_setup on that GPU, with
// that GPU current. Host code uses that address, never the array's name.
constexpr size_t kScratchDoubles = 65536 + 256;
__device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mutex;

mg_status init_scratch(mg_handle* h) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (h->device < 0 || h->device >= kMaxDevices)
        return fail(h, MG_ERR_ARG, "device %d out of range", h->device);
    if (!g_scratch[h->device]) {
        void* p = nullptr;
        HIP_TRY(h, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch[h->device] = static_cast<double*>(p);
    }
    return MG_OK;
}

// The work buffers a solve in the handle's precision uses, allocated ahead
// of the first solve (mg_setup, mg_set_options), so that a solve itself need
// not allocate.
mg_status ensure_buffers(mg_handle* h) {
    if (h->opt.precision == MG_PREC_FP64) return ensure_work<double>(h);
    MG_TRY(ensure_work<float>(h));
    if (h->opt.precision == MG_PREC_FP32 && !h->b32) {
        const long long n = h->lv[0].n;
        MG_TRY(dalloc(h, &h->b32, n));
        MG_TRY(dalloc(h, &h->u32a, n));
        MG_TRY(dalloc(h, &h->u32b, n));
    }
    return MG_OK;
}

// Forward or adjoint solve in the handle's precision; a mixed solve that
// stalls continues in FP64 (when fallback is allowed).
mg_status solve_in_precision(mg_handle* h, const double* rhs, double* u, double tol,
                             mg_stats* st, bool transposed, bool fallback) {
    const bool zero = h->opt.zero_guess != 0;
    if (h->opt.precision == MG_PREC_FP64)
        return outer<double, double>(h, rhs, u, tol, st, transposed, zero);
    if (h->opt.precision == MG_PREC_FP32)
        return outer<float, float>(h, rhs, u, tol, st, transposed, zero);
    mg_stats s1{};
    bool stalled = false;
    mg_status s = outer<float, double>(h, rhs, u, tol, &s1, transposed, zero,
                                       fallback ? &stalled : nullptr);
    if (s == MG_OK && stalled) {
        // the FP32 cycle stopped contracting: continue from the current
        // iterate (in u) with FP64 cycles for the remaining iterations
        mg_stats s2{};
        const int cap = h->opt.max_iters;
        h->opt.max_iters = cap - s1.iters;
        s = outer<double, double>(h, rhs, u, tol, &s2, transposed, false);
        h->opt.max_iters = cap;
        for (int m = 1; m <= s2.iters && s1.iters + m < MG_HIST; ++m)
            s1.res_hist[s1.iters + m] = s2.res_hist[m];
        s1.iters += s2.iters;
        s1.relres = s2.relres;
        s1.ms_total += s2.ms_total;
        s1.ms_vcycle += s2.ms_vcycle;
        s1.ms_residual += s2.ms_residual;
        s1.alg_bytes += s2.alg_bytes;
        for (int c = 0; c < MG_NK; ++c) {
            s1.kern_ms[c] += s2.kern_ms[c];
            s1.kern_launches[c] += s2.kern_launches[c];
            s1.kern_bytes[c] += s2.kern_bytes[c];
            s1.kern_fine_ms[c] += s2.kern_fine_ms[c];
            s1.kern_fine_launches[c] += s2.kern_fine_launches[c];
            s1.kern_fine_bytes[c] += s2.kern_fine_bytes[c];
        }
        s1.fell_back_fp64 = 1;
    }
    if (st) *st = s1;
    return s;
}

mg_status check_solve_args(mg_handle* h, const double* rhs, const double* u, double tol) {
    if (!rhs || !u) return fail(h, MG_ERR_ARG, "NULL field pointer");
    if (!(tol > 0) || !std::isfinite(tol)) return fail(h, MG_ERR_ARG, "tol must be > 0");
    if (rhs == u) return fail(h, MG_ERR_ARG, "rhs and solution must not alias");
    return MG_OK;
}

}  // namespace

// --- C ABI ---------------------------------------------------------------------
extern "C" {

void mg_options_default(mg_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->levels = 0;
    o->nu_pre = 2;
    o->nu_post = 2;
    o->coarse_sweeps = 40;
    o->max_iters = 100;
    o->omega = 0.8;
    o->semi_threshold = 2.0;
    o->precision = MG_PREC_MIXED;
    o->stream = nullptr;
    o->profile = 0;
    o->smooth_lo = 1.0 / 3.0;
    o->smooth_hi = 2.0;
    o->staged_columns = 65536;
    o->stall_factor = 0.9;
    o->stall_iters = 3;
    o->graphs = 1;
    o->zero_guess = 0;
    o->poison = 0;
}

mg_status mg_setup(const mg_grid* grid, const mg_coeffs* coeffs, const mg_options* opts,
                   mg_handle** out) {
    if (!out) return MG_ERR_ARG;
    *out = nullptr;
    if (!grid || !coeffs || !coeffs->alpha || !opts) return MG_ERR_ARG;
    std::string e = mgs::validate(*grid, *opts);
    if (!e.empty()) return MG_ERR_ARG;
    mg_handle* h = new (std::nothrow) mg_handle();
    if (!h) return MG_ERR_OOM;
    h->grid = *grid;
    h->opt = *opts;
    h->stream = static_cast<hipStream_t>(opts->stream);
    {
        const char* lg = std::getenv("MG_LOG");
        h->log = lg && *lg && std::strcmp(lg, "0") != 0;
    }
    mg_status s = hipGetDevice(&h->device) == hipSuccess ? MG_OK : MG_ERR_HIP;
    if (s == MG_OK) s = init_scratch(h);
    if (s == MG_OK) s = build(h, coeffs->alpha);
    if (s == MG_OK) s = ensure_buffers(h);
    if (s == MG_OK &&
        hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        h->cap_stream = nullptr;   // no graphs: direct launches
    }
    if (s == MG_OK) s = capture_graphs(h);
    if (s != MG_OK) {
        std::fprintf(stderr, "mg_setup: %s\n", h->err.c_str());
        release(h);
        delete h;
        return s;
    }
    *out = h;
    return MG_OK;
}

mg_status mg_update_coeffs(mg_handle* h, const mg_coeffs* coeffs) {
    if (!h) return MG_ERR_ARG;
    if (!coeffs || !coeffs->alpha) return fail(h, MG_ERR_ARG, "NULL coefficients");
    MG_TRY(set_coeffs(h, coeffs->alpha));
    // the graphs read the coefficients from the same buffers; only a change
    // of the coarsest route needs new ones
    if ((h->g32.exec && h->g32.dense_valid != h->dense.valid) ||
        (h->g64.exec && h->g64.dense_valid != h->dense.valid))
        return capture_graphs(h);
    return MG_OK;
}

mg_status mg_set_options(mg_handle* h, const mg_options* opts) {
    if (!h) return MG_ERR_ARG;
    if (!opts) return fail(h, MG_ERR_ARG, "NULL options");
    std::string e = mgs::validate(h->grid, *opts);
    if (!e.empty()) return fail(h, MG_ERR_ARG, "%s", e.c_str());
    if (opts->levels != h->opt.levels || opts->semi_threshold != h->opt.semi_threshold)
        return fail(h, MG_ERR_ARG, "levels and semi_threshold are fixed at setup");
    const bool recoarse = opts->coarse_sweeps != h->dense.sweeps || opts->omega != h->dense.omega;
    // the captured coarse V-cycle depends on these options only (not on the
    // stream, the stopping rule, profiling or the initial guess)
    const mg_options& o = h->opt;
    const bool recapture =
        opts->nu_pre != o.nu_pre || opts->nu_post != o.nu_post ||
        opts->coarse_sweeps != o.coarse_sweeps || opts->omega != o.omega ||
        opts->precision != o.precision || opts->smooth_lo != o.smooth_lo ||
        opts->smooth_hi != o.smooth_hi || opts->staged_columns != o.staged_columns ||
        opts->graphs != o.graphs;
    h->opt = *opts;
    h->stream = static_cast<hipStream_t>(opts->stream);
    MG_TRY(ensure_buffers(h));
    if (recoarse && h->dense.enabled) {
        MG_TRY(rebuild_dense(h));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    return recapture ? capture_graphs(h) : MG_OK;
}

static mg_status solve_common(mg_handle* h, const double* rhs, double* u, double tol,
                              mg_stats* st, bool transposed) {
    if (!h) return MG_ERR_ARG;
    MG_TRY(check_solve_args(h, rhs, u, tol));
    return solve_in_precision(h, rhs, u, tol, st, transposed, true);
}

mg_status mg_solve(mg_handle* h, const double* rhs, double* u, double tol, mg_stats* st) {
    return solve_common(h, rhs, u, tol, st, false);
}

mg_status mg_solve_adjoint(mg_handle* h, const double* w, double* lambda, double tol,
                           mg_stats* st) {
    return solve_common(h, w, lambda, tol, st, true);
}

mg_status mg_solve_noalloc(mg_handle* h, const double* rhs, double* u, double tol,
                           mg_stats* st) {
    if (!h) return MG_ERR_ARG;
    MG_TRY(check_solve_args(h, rhs, u, tol));
    double* sp = (h->device >= 0 && h->device < kMaxDevices) ? g_scratch[h->device] : nullptr;
    if (!sp) return fail(h, MG_ERR_ARG, "no scratch address for device %d", h->device);
    const size_t need = 2 * size_t(h->max_partials) + 2;
    if (need > kScratchDoubles)
        return fail(h, MG_ERR_ARG,
                    "grid too large for mg_solve_noalloc: %zu scratch values needed, %zu "
                    "available", need, kScratchDoubles);
    const bool ready = h->opt.precision == MG_PREC_FP64 ? h->have64
                       : h->opt.precision == MG_PREC_FP32 ? (h->have32 && h->b32)
                                                          : h->have32;
    if (!ready)
        return fail(h, MG_ERR_ARG, "the work buffers of this precision are not allocated");
    // run on the scratch, with no events and no profiling; restore after
    double* partials = h->partials;
    double* scalar = h->scalar;
    const int profile = h->opt.profile;
    h->partials = sp;
    h->scalar = sp + 2 * size_t(h->max_partials);
    h->no_events = true;
    h->no_graphs = true;
    h->opt.profile = 0;
    mg_status s = solve_in_precision(h, rhs, u, tol, st, false, h->have64);
    h->partials = partials;
    h->scalar = scalar;
    h->no_events = false;
    h->no_graphs = false;
    h->opt.profile = profile;
    return s;
}

mg_status mg_grad_alpha(mg_handle* h, const double* lambda, const double* u, double* g) {
    if (!h) return MG_ERR_ARG;
    if (!lambda || !u || !g) return fail(h, MG_ERR_ARG, "NULL field pointer");
    DevLevel& d = h->lv[0];
    mgk::grad_alpha(view<double>(d), d.V64, lambda, u, g, h->stream);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_launch(h, "grad_alpha");
}

mg_status mg_apply(mg_handle* h, const double* x, double* y) {
    if (!h) return MG_ERR_ARG;
    if (!x || !y || x == y) return fail(h, MG_ERR_ARG, "bad field pointers");
    DevLevel& d = h->lv[0];
    mgk::apply<double>(view<double>(d), x, nullptr, y, h->stream);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_launch(h, "apply");
}

mg_status mg_cell_volumes(mg_handle* h, double* V) {
    if (!h) return MG_ERR_ARG;
    if (!V) return fail(h, MG_ERR_ARG, "NULL field pointer");
    DevLevel& d = h->lv[0];
    mgk::cell_volumes(view<double>(d), d.V64, V, h->stream);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return check_launch(h, "cell_volumes");
}

mg_status mg_vcycle(mg_handle* h, const double* f, double* x, int32_t transposed) {
    if (!h) return MG_ERR_ARG;
    if (!f || !x || f == x) return fail(h, MG_ERR_ARG, "bad field pointers");
    prof_reset(h);
    if (h->opt.precision == MG_PREC_FP64) return one_vcycle<double>(h, f, x, transposed != 0);
    return one_vcycle<float>(h, f, x, transposed != 0);
}

mg_status mg_level_shape(const mg_handle* h, int32_t l, int32_t shape[3]) {
    if (!shape_ok(h, l) || !shape) return MG_ERR_ARG;
    shape[0] = h->lv[l].nI;
    shape[1] = h->lv[l].nJ;
    shape[2] = h->lv[l].nz;
    return MG_OK;
}

mg_status mg_level_sweep(mg_handle* h, int32_t l, const double* f, const double* x_in,
                         double* x_out) {
    if (!h) return MG_ERR_ARG;
    if (!shape_ok(h, l) || !f || !x_out) return fail(h, MG_ERR_ARG, "bad level or pointer");
    prof_reset(h);
    if (h->opt.precision == MG_PREC_FP64) return level_sweep<double>(h, l, f, x_in, x_out);
    return level_sweep<float>(h, l, f, x_in, x_out);
}

mg_status mg_level_residual_restrict(mg_handle* h, int32_t l, const double* f,
                                     const double* x, double* fc) {
    if (!h) return MG_ERR_ARG;
    if (!shape_ok(h, l + 1) || l < 0 || !f || !fc)
        return fail(h, MG_ERR_ARG, "bad level or pointer");
    prof_reset(h);
    if (h->opt.precision == MG_PREC_FP64) return level_restrict<double>(h, l, f, x, fc);
    return level_restrict<float>(h, l, f, x, fc);
}

mg_status mg_level_prolong_add(mg_handle* h, int32_t l, const double* xc, double* x) {
    if (!h) return MG_ERR_ARG;
    if (!shape_ok(h, l + 1) || l < 0 || !xc || !x)
        return fail(h, MG_ERR_ARG, "bad level or pointer");
    prof_reset(h);
    if (h->opt.precision == MG_PREC_FP64) return level_prolong<double>(h, l, xc, x);
    return level_prolong<float>(h, l, xc, x);
}

mg_status mg_plan(const mg_grid* grid, const mg_options* opts, int32_t* levels_out,
                  int32_t* nlon_out, int32_t* nlat_out, int32_t* child_first,
                  int32_t* child_count, int32_t cap) {
    if (!grid || !opts || !levels_out || !nlon_out || !nlat_out) return MG_ERR_ARG;
    if (!mgs::validate(*grid, *opts).empty()) return MG_ERR_ARG;
    mgs::Hierarchy H;
    if (!mgs::plan(*grid, opts->levels, opts->semi_threshold, H).empty()) return MG_ERR_ARG;
    *levels_out = int32_t(H.levels.size());
    int32_t pos = 0;
    for (size_t l = 0; l < H.levels.size(); ++l) {
        nlon_out[l] = H.levels[l].nI;
        nlat_out[l] = H.levels[l].nJ;
        if (l == 0) continue;
        for (int J = 0; J < H.levels[l].nJ; ++J) {
            if (child_first && child_count) {
                if (pos >= cap) return MG_ERR_ARG;
                child_first[pos] = H.levels[l].child_first[J];
                child_count[pos] = H.levels[l].child_count[J];
            }
            ++pos;
        }
    }
    return MG_OK;
}

mg_status mg_plan_tables(const mg_grid* grid, const mg_options* opts, int32_t l, double* V,
                         double* Tlam, double* Tth, double* Tr) {
    if (!grid || !opts) return MG_ERR_ARG;
    if (!mgs::validate(*grid, *opts).empty()) return MG_ERR_ARG;
    mgs::Hierarchy H;
    if (!mgs::plan(*grid, opts->levels, opts->semi_threshold, H).empty()) return MG_ERR_ARG;
    if (l < 0 || l >= int(H.levels.size())) return MG_ERR_ARG;
    const mgs::Level& s = H.levels[l];
    if (V) std::copy(s.V.begin(), s.V.end(), V);
    if (Tlam) std::copy(s.Tlam.begin(), s.Tlam.end(), Tlam);
    if (Tth) std::copy(s.Tth.begin(), s.Tth.end(), Tth);
    if (Tr) std::copy(s.Tr.begin(), s.Tr.end(), Tr);
    return MG_OK;
}

void mg_destroy(mg_handle* h) {
    if (!h) return;
    release(h);
    delete h;
}

const char* mg_status_string(mg_status s) {
    switch (s) {
        case MG_OK: return "ok";
        case MG_ERR_NOT_CONVERGED: return "not converged";
        case MG_ERR_ARG: return "invalid argument";
        case MG_ERR_HIP: return "HIP runtime error";
        case MG_ERR_OOM: return "out of device memory";
        case MG_ERR_BREAKDOWN: return "breakdown (non-finite residual)";
    }
    return "unknown status";
}

const char* mg_last_error(const mg_handle* h) { return h ? h->err.c_str() : ""; }

}  // extern "C"
