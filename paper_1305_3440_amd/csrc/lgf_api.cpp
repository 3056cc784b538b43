// lgf_api.cpp -- the C ABI of include/lgf.h: handles, device memory, the
// canonical-array boundary, and the gauge-fixing driver (Sec. 4 of Schroeck
// and Vogt, arXiv:1305.3440: sweep the two parities in turn until theta
// reaches the target), with the mixed FP32-bulk / FP64-finish policy,
// hipGraph-captured sweep chunks and the sweep-kernel autotuner.
#include "lgf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lgf_device.hpp"
#include "lgf_host.hpp"
#include "lgf_internal.hpp"

namespace lgf {

namespace {
thread_local std::string g_last_error;
}

lgf_status fail(lgf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

const char *last_error() { return g_last_error.c_str(); }

bool valid_format(int f) { return f >= LGF_FP64_18 && f <= LGF_FP64_12; }

bool valid_dims(const int dims[4])
{
    if (!dims) return false;
    uint64_t V = 1;
    for (int d = 0; d < 4; ++d) {
        if (dims[d] < 2 || (dims[d] & 1)) return false;
        V *= (uint64_t)dims[d];
    }
    return V <= (1ull << 31);
}

Geom make_geom(const int dims[4])
{
    Geom g;
    for (int d = 0; d < 4; ++d) g.L[d] = (uint32_t)dims[d];
    g.hx = g.L[3] / 2;
    g.Vh = g.L[0] * g.L[1] * g.L[2] * g.hx;
    g.hs[0] = g.L[1] * g.L[2] * g.hx;
    g.hs[1] = g.L[2] * g.hx;
    g.hs[2] = g.hx;
    return g;
}

double elapsed_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return (double)ms;
}

}  // namespace lgf

namespace {

using lgf::fail;
using lgf::valid_format;
using lgf::valid_dims;
using lgf::make_geom;
using lgf::elapsed_ms;

struct GraphEntry {
    int format;
    void *field;
    int n_sweeps;
    double omega;
    lgf::SweepTuning tune;
    int coulomb;
    void *gacc;
    int fused;
    double p_sr;
    uint64_t seed;
    int fixed;  // fixed-link form: field holds the links, gacc the gauge transformation
    hipGraphExec_t exec;
};

bool same_chunk(const GraphEntry &a, const GraphEntry &b, bool sr)
{
    return a.format == b.format && a.field == b.field && a.n_sweeps == b.n_sweeps && a.omega == b.omega &&
           a.tune == b.tune && a.coulomb == b.coulomb && a.gacc == b.gacc && a.fused == b.fused &&
           a.p_sr == b.p_sr && (!sr || a.seed == b.seed) && a.fixed == b.fixed;
}

constexpr int64_t kStageSites = 1 << 16;  // sites per canonical staging chunk (37.7 MB)

}  // namespace

struct lgf_lattice {
    int dims[4];
    int64_t V;
    lgf::Geom geom;
    int format;
    void *field;
    size_t field_bytes;
    bool owned;
    hipStream_t stream;
    bool own_stream;
    int device;
    double *d_partials;
    double *d_out;
    double *h_out;  // pinned, 2 doubles
    double *d_stage;
    int64_t *d_sites;
    int64_t sites_cap;
    void *work[4];  // owned per-format copies for the mixed-precision bulk
    size_t work_bytes[4];
    void *partner[4];  // owned second buffer per format for the out-of-place schedule
    double *d_fused;   // partial sums of the measurement fused into a sweep
    size_t fused_cap;  // (F, theta) pairs d_fused holds
    uint64_t *d_sweep_base;               // device copy of a chunk's first SR counter
    const uint64_t *sweep_base_active;    // passed to the sweeps while a chunk is captured
    lgf::SweepTuning tune[4];
    std::vector<GraphEntry> graphs;
    hipEvent_t ev0, ev1;
    // Coulomb gauge: timeslice flags and per-timeslice reductions (lazily)
    uint8_t *d_mask;
    uint8_t *h_mask;   // pinned, Lt flags
    double *d_cpart;
    double *d_cout;
    double *h_cout;    // pinned, 2 Lt doubles
    // accumulated gauge transformation of the mixed-precision bulk
    void *gacc;        // site field in the bulk format (owned), or NULL
    size_t gacc_bytes;
    void *gacc_active; // passed to the sweeps while the bulk accumulates
    // fixed-link form: the gauge transformation per sweep format (owned site
    // fields) and the tuning of its sweep
    void *gfix[4];
    lgf::SweepTuning tune_fixed[5];  // per sweep format, LGF_FP64_12S included
    void *split;       // the links in the split storage of LGF_FP64_12S (owned)
    void *rec[5];      // per-site link records of the 12-real formats (owned)
    // stepwise fixed-link gauge fixing (lgf_fix_begin .. lgf_fix_end)
    bool fix_on;
    int fix_format;
    const void *fix_links;
    // accept-reject trial counter of the annealing sweeps (lazily)
    unsigned long long *d_trials;
};

namespace {

lgf_status use_device(const lgf_lattice *h)
{
    int cur = -1;
    LGF_HIP(hipGetDevice(&cur));
    if (cur != h->device) LGF_HIP(hipSetDevice(h->device));
    return LGF_OK;
}

void drop_graphs(lgf_lattice *h)
{
    for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

lgf_status ensure_stage(lgf_lattice *h)
{
    if (!h->d_stage) {
        const int64_t n = h->V < kStageSites ? h->V : kStageSites;
        LGF_HIP(hipMalloc(&h->d_stage, (size_t)n * 72 * sizeof(double)));
    }
    return LGF_OK;
}

lgf_status ensure_sites(lgf_lattice *h, int64_t n)
{
    if (h->sites_cap < n) {
        if (h->d_sites) LGF_HIP(hipFree(h->d_sites));
        h->d_sites = nullptr;
        h->sites_cap = 0;
        LGF_HIP(hipMalloc(&h->d_sites, (size_t)n * sizeof(int64_t)));
        h->sites_cap = n;
    }
    return LGF_OK;
}

lgf_status ensure_work(lgf_lattice *h, int format)
{
    if (!h->work[format]) {
        const size_t bytes = (size_t)h->V * 4 * lgf::link_bytes(format);
        hipError_t e = hipMalloc(&h->work[format], bytes);
        if (e != hipSuccess) {
            h->work[format] = nullptr;
            (void)hipGetLastError();
            return fail(LGF_ENOMEM, "cannot allocate %zu bytes for the %d-format copy", bytes, format);
        }
        h->work_bytes[format] = bytes;
    }
    return LGF_OK;
}

// The accumulated gauge transformation of an FP32 bulk (a site field in the
// bulk format): allocated once, set to the identity here and handed to the
// sweeps, which multiply in every update's G.
lgf_status gacc_begin(lgf_lattice *h, int bulk)
{
    const size_t gbytes = (size_t)h->V * lgf::link_bytes(bulk);
    if (h->gacc && h->gacc_bytes != gbytes) {
        (void)hipFree(h->gacc);
        h->gacc = nullptr;
    }
    if (!h->gacc) {
        if (hipMalloc(&h->gacc, gbytes) != hipSuccess) {
            h->gacc = nullptr;
            (void)hipGetLastError();
            return fail(LGF_ENOMEM, "cannot allocate %zu bytes for the accumulated gauge field", gbytes);
        }
        h->gacc_bytes = gbytes;
    }
    LGF_HIP(lgf::launch_site_field(bulk, h->gacc, h->geom, 0, h->stream));
    h->gacc_active = h->gacc;
    return LGF_OK;
}

// End the accumulation: dst (format fd) <- g(x) U(x) g(x+mu)^dag from the
// handle's untouched FP64 field, each g reunitarized in FP64 first -- an exact
// gauge transformation of the input.
lgf_status gacc_apply(lgf_lattice *h, int bulk, int fd, void *dst)
{
    h->gacc_active = nullptr;
    LGF_HIP(lgf::launch_gauge_transform(h->format, h->field, bulk, h->gacc, fd, dst, h->geom, h->stream));
    return LGF_OK;
}

// the second buffer of a format's out-of-place sweep (a whole field's size)
lgf_status ensure_partner(lgf_lattice *h, int format)
{
    if (!h->partner[format]) {
        const size_t bytes = (size_t)h->V * 4 * lgf::link_bytes(format);
        if (hipMalloc(&h->partner[format], bytes) != hipSuccess) {
            h->partner[format] = nullptr;
            (void)hipGetLastError();
            return fail(LGF_ENOMEM, "cannot allocate %zu bytes for the out-of-place partner buffer", bytes);
        }
    }
    return LGF_OK;
}

// The starting tuning of a format: one lane per site, 128-lane workgroups,
// non-temporal access; the FP64 12-real sweep of the mixed finish out of place
// (on every GPU measured within a few per cent of the fastest variant, often
// the fastest), the others in place.
lgf::SweepTuning default_tuning(int format)
{
    lgf::SweepTuning t{};
    if (format == LGF_FP64_12) t.schedule = lgf::kScheduleOutOfPlace;
    return t;
}

// Before sweeps in a format: the out-of-place schedule needs its partner
// buffer (allocated here, never inside a graph capture); without memory for
// it the format falls back to in place.
void prepare_schedule(lgf_lattice *h, int format)
{
    if (h->tune[format].schedule != lgf::kScheduleOutOfPlace || h->partner[format]) return;
    if (ensure_partner(h, format) != LGF_OK) {
        h->tune[format].schedule = lgf::kScheduleInPlace;
        drop_graphs(h);
    }
}

// F and theta of a field; with reunit the links are first projected onto
// SU(3) in FP64 (fused: parity 0 reunitarizes its forward links and, in
// registers, its backward links; parity 1 then reads the already stored ones).
lgf_status measure_field(lgf_lattice *h, int format, void *field, bool reunit, double *F, double *theta)
{
    int n0 = 0, n1 = 0;
    LGF_HIP(lgf::launch_measure(format, field, h->geom, 0, reunit, reunit, h->d_partials, &n0, h->stream));
    LGF_HIP(lgf::launch_measure(format, field, h->geom, 1, reunit, false, h->d_partials + 2 * n0, &n1,
                                h->stream));
    LGF_HIP(lgf::launch_finish_measure(h->d_partials, n0 + n1, (double)h->V, h->d_out, h->stream));
    LGF_HIP(hipMemcpyAsync(h->h_out, h->d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    if (F) *F = h->h_out[0];
    if (theta) *theta = h->h_out[1];
    return LGF_OK;
}

lgf_status sweep_launch(lgf_lattice *h, int format, void *field, int parity, double omega, double p_sr,
                        uint64_t seed, uint64_t sweep_index, bool coulomb = false, double *meas = nullptr)
{
    lgf::SweepArgs a{parity, omega, p_sr, seed, sweep_index, 0u};
    a.gacc = h->gacc_active;
    a.meas = meas;
    a.sweep_base = h->sweep_base_active;
    if (coulomb)
        LGF_HIP(lgf::launch_sweep_coulomb(format, field, h->geom, a, h->d_mask, h->tune[format].nontemporal != 0,
                                          h->stream));
    else
        LGF_HIP(lgf::launch_sweep(format, field, h->geom, a, h->tune[format], h->stream));
    return LGF_OK;
}

// One full sweep (parity 0, then parity 1).  With the pipeline tuning the
// sweep is issued slice by slice in t: parity 0 of slice k, then parity 1 of
// slice k-1, whose neighbours in slices k-2, k-1, k are all done by then;
// parity 1 of slices Lt-1 and 0 (which needs slice Lt-1) close the sweep.
// Every site update sees the same links as in the two-launch order, so the
// result is the same bit for bit, while parity 1 finds the links parity 0
// wrote one slice earlier still in the last-level cache.
// meas: the parity-1 half-sweep also reunitarizes the links it writes and
// leaves its (F, theta) partial sums there (see measure_fused).
lgf_status full_sweep(lgf_lattice *h, int format, void *field, double omega, double p_sr, uint64_t seed,
                      uint64_t sweep_index, bool coulomb = false, double *meas = nullptr)
{
    const int Lt = h->dims[0];
    const int sched = h->tune[format].schedule;
    if (!coulomb && sched == lgf::kScheduleOutOfPlace) {
        // parity 0 moves every link into the partner buffer, parity 1 moves them back
        void *partner = h->partner[format];
        if (!partner || partner == field) return fail(LGF_ESTATE, "no partner buffer for the out-of-place sweep");
        lgf::SweepArgs a{0, omega, p_sr, seed, sweep_index, 0u};
        a.gacc = h->gacc_active;
        a.sweep_base = h->sweep_base_active;
        a.out = partner;
        LGF_HIP(lgf::launch_sweep(format, field, h->geom, a, h->tune[format], h->stream));
        a.parity = 1;
        a.out = field;
        a.meas = meas;
        LGF_HIP(lgf::launch_sweep(format, partner, h->geom, a, h->tune[format], h->stream));
        return LGF_OK;
    }
    // (the pipeline gives the two-launch result bit for bit, so a sweep that
    // carries the fused measurement simply runs as two launches)
    if (coulomb || sched != lgf::kSchedulePipeline || Lt < 4 || meas) {
        LGF_TRY(sweep_launch(h, format, field, 0, omega, p_sr, seed, sweep_index, coulomb));
        LGF_TRY(sweep_launch(h, format, field, 1, omega, p_sr, seed, sweep_index, coulomb, meas));
        return LGF_OK;
    }
    const uint32_t hs = h->geom.hs[0];
    auto slice = [&](int parity, int t) -> lgf_status {
        lgf::SweepArgs a{parity, omega, p_sr, seed, sweep_index, 0u};
        a.gacc = h->gacc_active;
        a.sweep_base = h->sweep_base_active;
        a.h_begin = (uint32_t)t * hs;
        a.h_end = (uint32_t)(t + 1) * hs;
        LGF_HIP(lgf::launch_sweep(format, field, h->geom, a, h->tune[format], h->stream));
        return LGF_OK;
    };
    LGF_TRY(slice(0, 0));
    LGF_TRY(slice(0, 1));
    for (int k = 2; k < Lt; ++k) {
        LGF_TRY(slice(0, k));
        LGF_TRY(slice(1, k - 1));
    }
    LGF_TRY(slice(1, Lt - 1));
    LGF_TRY(slice(1, 0));
    return LGF_OK;
}

// Coulomb-gauge scratch: timeslice flags and per-timeslice partial sums
lgf_status ensure_coulomb(lgf_lattice *h)
{
    if (h->d_mask) return LGF_OK;
    const int Lt = h->dims[0];
    // room for the link form's and the fixed-link form's partial sums
    const size_t bps = (size_t)std::max(lgf::coulomb_blocks_per_slice(h->geom), lgf::coulomb_fixed_blocks(h->geom));
    const size_t parts = (size_t)4 * Lt * bps;
    hipError_t e;
    if ((e = hipMalloc(&h->d_mask, Lt)) != hipSuccess ||
        (e = hipHostMalloc((void **)&h->h_mask, Lt, hipHostMallocDefault)) != hipSuccess ||
        (e = hipMalloc(&h->d_cpart, parts * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&h->d_cout, 2 * Lt * sizeof(double))) != hipSuccess ||
        (e = hipHostMalloc((void **)&h->h_cout, 2 * Lt * sizeof(double), hipHostMallocDefault)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LGF_ENOMEM, "Coulomb scratch allocation failed: %s", hipGetErrorString(e));
    }
    return LGF_OK;
}

// copy the host flags (NULL = all active) to the device mask; synchronises
lgf_status upload_mask(lgf_lattice *h, const unsigned char *flags)
{
    for (int t = 0; t < h->dims[0]; ++t) h->h_mask[t] = flags ? (flags[t] ? 1 : 0) : 1;
    LGF_HIP(hipMemcpyAsync(h->d_mask, h->h_mask, h->dims[0], hipMemcpyHostToDevice, h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    return LGF_OK;
}

// per-timeslice F_C(t), theta_C(t) into h->h_cout (2 Lt doubles); with reunit
// the fused FP64 reunitarization of every link first
lgf_status measure_coulomb_field(lgf_lattice *h, int format, void *field, bool reunit)
{
    const size_t half = (size_t)2 * h->dims[0] * lgf::coulomb_blocks_per_slice(h->geom);
    LGF_HIP(lgf::launch_measure_coulomb(format, field, h->geom, 0, reunit, reunit, h->d_cpart, h->stream));
    LGF_HIP(lgf::launch_measure_coulomb(format, field, h->geom, 1, reunit, false, h->d_cpart + half, h->stream));
    LGF_HIP(lgf::launch_finish_coulomb(h->d_cpart, h->geom, lgf::coulomb_blocks_per_slice(h->geom), h->d_cout,
                                       h->stream));
    LGF_HIP(hipMemcpyAsync(h->h_cout, h->d_cout, 2 * h->dims[0] * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    return LGF_OK;
}

// n full sweeps on (format, field).  Overrelaxation chunks (no random
// numbers, so every launch of the chunk has fixed arguments) are captured once
// into a hipGraph and replayed; stochastic relaxation launches directly since
// its counter changes every sweep.
// Whether the chunk's last half-sweep can carry the reunitarization and the
// measurement (kernel variants exist for overrelaxation with non-temporal
// access, Landau gauge).
bool can_fuse(const lgf_lattice *h, int format, double p_sr, bool coulomb)
{
    return !coulomb && p_sr == 0.0 && h->tune[format].nontemporal != 0;
}

// room for the fused sweep's partial sums followed by those of the parity-0
// measurement pass; graphs that hold the old buffer are dropped on growth
lgf_status ensure_fused_cap(lgf_lattice *h, size_t need)
{
    if (h->fused_cap >= need) return LGF_OK;
    drop_graphs(h);
    if (h->d_fused) LGF_HIP(hipFree(h->d_fused));
    h->d_fused = nullptr;
    h->fused_cap = 0;
    if (hipMalloc(&h->d_fused, need * 2 * sizeof(double)) != hipSuccess) {
        h->d_fused = nullptr;
        (void)hipGetLastError();
        return fail(LGF_ENOMEM, "cannot allocate the fused measurement's partial sums");
    }
    h->fused_cap = need;
    return LGF_OK;
}

lgf_status ensure_fused(lgf_lattice *h, int format)
{
    return ensure_fused_cap(h, (size_t)lgf::sweep_groups(h->geom, h->tune[format]) +
                                   (size_t)lgf::measure_blocks(h->geom));
}

// F and theta after a chunk whose last half-sweep was fused: its partial sums
// (parity-1 sites' theta, parity-1 forward links' Re tr, from the links as
// reunitarized and stored) plus a read-only pass over the parity-0 sites.
lgf_status measure_fused(lgf_lattice *h, int format, void *field, double *F, double *theta)
{
    const int ng = (int)lgf::sweep_groups(h->geom, h->tune[format]);
    int n0 = 0;
    LGF_HIP(lgf::launch_measure(format, field, h->geom, 0, false, false, h->d_fused + 2 * (size_t)ng, &n0,
                                h->stream));
    LGF_HIP(lgf::launch_finish_measure(h->d_fused, ng + n0, (double)h->V, h->d_out, h->stream));
    LGF_HIP(hipMemcpyAsync(h->h_out, h->d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    if (F) *F = h->h_out[0];
    if (theta) *theta = h->h_out[1];
    return LGF_OK;
}

// Launch the chunk of sweeps that issue() enqueues through a hipGraph: the
// cached graph with the same key is replayed, otherwise issue() is captured
// into a new one (at most 8 kept).  For stochastic relaxation the captured
// launches carry counter offsets and read the chunk's first counter from
// h->d_sweep_base, written here before the replay.
template <class Issue>
lgf_status run_captured(lgf_lattice *h, const GraphEntry &key, uint64_t sweep0, Issue issue)
{
    const bool sr = key.p_sr > 0.0;
    if (sr) LGF_HIP(lgf::launch_set_u64(h->d_sweep_base, sweep0, h->stream));
    for (auto &g : h->graphs) {
        if (same_chunk(g, key, sr)) {
            LGF_HIP(hipGraphLaunch(g.exec, h->stream));
            return LGF_OK;
        }
    }
    hipGraph_t graph = nullptr;
    LGF_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    h->sweep_base_active = sr ? h->d_sweep_base : nullptr;
    const lgf_status st = issue();
    h->sweep_base_active = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &graph);
    if (st != LGF_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(LGF_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(LGF_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    if (h->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(h->graphs.front().exec);
        h->graphs.erase(h->graphs.begin());
    }
    GraphEntry entry = key;
    entry.exec = exec;
    h->graphs.push_back(entry);
    LGF_HIP(hipGraphLaunch(exec, h->stream));
    return LGF_OK;
}

// fused: the last sweep reunitarizes and measures (see measure_fused); the
// caller checked can_fuse
lgf_status run_chunk(lgf_lattice *h, int format, void *field, int n, double omega, double p_sr,
                     uint64_t seed, uint64_t sweep0, bool use_graph, bool coulomb = false, bool fused = false)
{
    if (!coulomb) prepare_schedule(h, format);
    if (fused) LGF_TRY(ensure_fused(h, format));
    auto meas_of = [&](int k) { return (fused && k == n - 1) ? h->d_fused : nullptr; };
    if (!use_graph) {
        for (int k = 0; k < n; ++k)
            LGF_TRY(full_sweep(h, format, field, omega, p_sr, seed, sweep0 + (uint64_t)k, coulomb, meas_of(k)));
        return LGF_OK;
    }
    // stochastic relaxation: the captured sweeps carry counter offsets 0..n-1
    // and read the chunk's first counter from the device, set here outside
    // the graph, so one graph serves every chunk
    const bool sr = p_sr > 0.0;
    GraphEntry key{format, field, n, omega, h->tune[format], coulomb ? 1 : 0, h->gacc_active, fused ? 1 : 0,
                   p_sr, seed, 0, nullptr};
    return run_captured(h, key, sweep0, [&]() -> lgf_status {
        for (int k = 0; k < n; ++k)
            LGF_TRY(full_sweep(h, format, field, omega, p_sr, seed, sr ? (uint64_t)k : sweep0 + (uint64_t)k,
                               coulomb, meas_of(k)));
        return LGF_OK;
    });
}

// The autotuners' search over `variants`: each timed once over `trials` full
// sweeps (stage 1), then the four fastest and the default again over ten times
// as many sweeps in five interleaved rounds; the smallest median wins, but a
// variant replaces the default only when at least 1 % faster (single short
// timings of variants a few per cent apart are within the run-to-run noise,
// and near-ties within what one GPU's timings drift over a long run).
// time_variant(tuning, n, &ms) times n full sweeps.  With LGF_AUTOTUNE_LOG
// set, the stage-2 medians go to stderr.  False when a timing failed.
template <class TimeFn>
bool pick_variant(const std::vector<lgf::SweepTuning> &variants, const lgf::SweepTuning &dflt, int trials,
                  const char *who, int format, TimeFn &&time_variant, lgf::SweepTuning *best)
{
    struct Cand {
        lgf::SweepTuning t;
        double ms;
    };
    std::vector<Cand> cands;
    for (const auto &t : variants) {
        Cand c{t, 0.0};
        if (!time_variant(t, trials, &c.ms)) return false;
        cands.push_back(c);
    }
    std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
    std::vector<lgf::SweepTuning> finals;
    for (size_t i = 0; i < cands.size() && finals.size() < 4; ++i) finals.push_back(cands[i].t);
    bool have_default = false;
    for (const auto &t : finals) have_default = have_default || t == dflt;
    if (!have_default) finals.push_back(dflt);
    std::vector<std::vector<double>> ms(finals.size());
    const int n2 = std::max(10 * trials, 20);
    for (int round = 0; round < 5; ++round)
        for (size_t i = 0; i < finals.size(); ++i) {
            double m = 0.0;
            if (!time_variant(finals[i], n2, &m)) return false;
            ms[i].push_back(m);
        }
    double best_ms = 1e300;
    const bool log = std::getenv("LGF_AUTOTUNE_LOG") != nullptr;
    for (size_t i = 0; i < finals.size(); ++i) {
        std::sort(ms[i].begin(), ms[i].end());
        if (log) {
            const lgf::SweepTuning &t = finals[i];
            std::fprintf(stderr, "%s format %d: lanes %d block %d xcd %d nt %d schedule %d spt %d: "
                         "median %.4f ms per full sweep (min %.4f, max %.4f)\n", who, format, t.lanes_per_site,
                         t.block, t.xcd_remap, t.nontemporal, t.schedule, t.sites_per_thread, ms[i][2], ms[i][0],
                         ms[i][4]);
        }
        if (ms[i][2] < best_ms) {
            best_ms = ms[i][2];
            *best = finals[i];
        }
    }
    for (size_t i = 0; i < finals.size(); ++i)
        if (finals[i] == dflt && best_ms > 0.99 * ms[i][2]) *best = dflt;
    return true;
}

// ----------------------------------------------------------------------------
// Fixed-link form: the links stay as they are and the sweeps update the gauge
// transformation g, a site field in the sweep's format.
// ----------------------------------------------------------------------------

// Lattices from this many sites on read per-site link records by default:
// measured faster from 24^4 up (FP64-12 4-6 % at 24^4 and 32^4), slower at
// 16^4, where a half-sweep takes about 10 us and the records' larger
// footprint costs more than their layout returns.
constexpr int64_t kRecordsMinSites = 1 << 18;

// Starting tuning of the fixed-link sweep (the fastest measured at 64^4):
// FP64-12 and the split links with 2 lanes per site (one lane runs one wave
// per SIMD in FP64) in 128-lane workgroups over the blocked tile order on
// per-site link records; FP32-12 with one lane per site in 128-lane
// workgroups, lexicographic, on records; FP64-18 with 2 lanes in 64-lane
// workgroups over the blocked tile order, FP32-18 with 2 lanes in 256-lane
// workgroups, lexicographic.  Below kRecordsMinSites sites the link field.
lgf::SweepTuning default_fixed_tuning(int format, int64_t V)
{
    lgf::SweepTuning t{};
    t.lanes_per_site = 2;
    const bool fp64 = (format == LGF_FP64_18 || format == LGF_FP64_12 || format == LGF_FP64_12S);
    t.block = fp64 ? 64 : 256;
    t.xcd_remap = fp64 ? 2 : 0;
    const int layout = (V >= kRecordsMinSites) ? lgf::kLayoutRecords : lgf::kLayoutPlanes;
    if (format == LGF_FP64_12 || format == LGF_FP64_12S) {
        t.block = 128;
        t.schedule = layout;
    } else if (format == LGF_FP32_12) {
        t.lanes_per_site = 1;
        t.block = 128;
        t.schedule = layout;
    }
    return t;
}

// format of the gauge transformation of a fixed-link sweep format (FP64-12
// for the split links) and its site field
int gf_format(int format) { return format == LGF_FP64_12S ? LGF_FP64_12 : format; }
void *gfix_of(lgf_lattice *h, int format) { return h->gfix[gf_format(format)]; }

bool valid_fixed_format(int f) { return valid_format(f) || f == LGF_FP64_12S; }

lgf_status ensure_gfix(lgf_lattice *h, int format)
{
    const int f = gf_format(format);
    if (!h->gfix[f]) {
        const size_t bytes = (size_t)h->V * lgf::link_bytes(f);
        if (hipMalloc(&h->gfix[f], bytes) != hipSuccess) {
            h->gfix[f] = nullptr;
            (void)hipGetLastError();
            return fail(LGF_ENOMEM, "cannot allocate %zu bytes for the gauge transformation", bytes);
        }
    }
    return LGF_OK;
}

// the links of the fixed-link sweeps in `format`: the handle's own field, or
// a copy of it in the working buffer of that format (LGF_FP64_12S: in the
// split storage)
lgf_status links_in_format(lgf_lattice *h, int format, void **links)
{
    if (format == LGF_FP64_12S) {
        if (!h->split) {
            const size_t bytes = lgf::split_links_bytes(h->geom);
            if (hipMalloc(&h->split, bytes) != hipSuccess) {
                h->split = nullptr;
                (void)hipGetLastError();
                return fail(LGF_ENOMEM, "cannot allocate %zu bytes for the split links", bytes);
            }
        }
        LGF_HIP(lgf::launch_split_links(h->format, h->field, h->split, h->geom, h->stream));
        *links = h->split;
        return LGF_OK;
    }
    if (format == h->format) {
        *links = h->field;
        return LGF_OK;
    }
    LGF_TRY(ensure_work(h, format));
    LGF_HIP(lgf::launch_convert(h->format, h->field, format, h->work[format], h->geom, false, h->stream));
    *links = h->work[format];
    return LGF_OK;
}

// whether the Landau fixed-link sweeps in `format` read per-site link records
bool fixed_records(const lgf_lattice *h, int format)
{
    return h->tune_fixed[format].schedule == lgf::kLayoutRecords;
}

// the per-site link records of format (a 12-real format) built from its link
// field, in h->rec[format]; false (and nothing built) without memory for them
lgf_status build_records(lgf_lattice *h, int format, bool *built)
{
    *built = false;
    void *planes = nullptr;
    LGF_TRY(links_in_format(h, format, &planes));
    if (!h->rec[format]) {
        const size_t bytes = lgf::record_links_bytes(format, h->geom);
        if (bytes == 0) return fail(LGF_EINVAL, "format %d has no per-site link records", format);
        if (hipMalloc(&h->rec[format], bytes) != hipSuccess) {
            h->rec[format] = nullptr;
            (void)hipGetLastError();
            return LGF_OK;
        }
    }
    LGF_HIP(lgf::launch_record_links(format, planes, h->rec[format], h->geom, h->stream));
    *built = true;
    return LGF_OK;
}

// the links of the Landau fixed-link sweeps in `format`, laid out as the
// format's tuning reads them: the link field (links_in_format) or its
// per-site records.  Without memory for the records the tuning falls back to
// the link field.
lgf_status fixed_links(lgf_lattice *h, int format, void **links)
{
    if (fixed_records(h, format)) {
        bool built = false;
        LGF_TRY(build_records(h, format, &built));
        if (built) {
            *links = h->rec[format];
            return LGF_OK;
        }
        h->tune_fixed[format].schedule = lgf::kLayoutPlanes;
        drop_graphs(h);
    }
    return links_in_format(h, format, links);
}

// n full sweeps in the fixed-link form.  The chunk's last sweep stores every g
// reunitarized (both half-sweeps); with fused, its parity-1 half-sweep also
// leaves the (F, theta) partial sums of its sites in h->d_fused.
lgf_status run_chunk_fixed(lgf_lattice *h, int format, const void *links, void *gf, int n, double omega,
                           double p_sr, uint64_t seed, uint64_t sweep0, bool use_graph, bool fused,
                           bool coulomb = false)
{
    const lgf::SweepTuning &t = h->tune_fixed[format];
    if (fused)
        LGF_TRY(ensure_fused_cap(h, (size_t)lgf::fixed_sweep_groups(h->geom, t) +
                                        (size_t)lgf::fixed_measure_blocks(h->geom)));
    const bool sr = p_sr > 0.0;
    auto issue = [&](bool captured) -> lgf_status {
        for (int k = 0; k < n; ++k) {
            const bool last = (k == n - 1);
            lgf::SweepArgs a{0, omega, p_sr, seed, (captured && sr) ? (uint64_t)k : sweep0 + (uint64_t)k, 0u};
            a.sweep_base = h->sweep_base_active;
            if (coulomb) {
                // timeslice flags read from the device at run time (set before the chunk)
                LGF_HIP(lgf::launch_fixed_sweep_coulomb(format, links, gf, h->geom, a, t, last ? 1 : 0, h->d_mask,
                                                        h->stream));
                a.parity = 1;
                LGF_HIP(lgf::launch_fixed_sweep_coulomb(format, links, gf, h->geom, a, t, last ? 1 : 0, h->d_mask,
                                                        h->stream));
                continue;
            }
            LGF_HIP(lgf::launch_fixed_sweep(format, links, gf, h->geom, a, t, last ? 1 : 0, h->stream));
            a.parity = 1;
            a.meas = (last && fused) ? h->d_fused : nullptr;
            LGF_HIP(lgf::launch_fixed_sweep(format, links, gf, h->geom, a, t, last ? (fused ? 2 : 1) : 0, h->stream));
        }
        return LGF_OK;
    };
    if (!use_graph) return issue(false);
    GraphEntry key{format, const_cast<void *>(links), n, omega, t, coulomb ? 1 : 0, gf, fused ? 1 : 0, p_sr, seed,
                   1, nullptr};
    return run_captured(h, key, sweep0, [&]() { return issue(true); });
}

// F and theta of the links g(x) U_mu(x) g(x+mu)^dag: after a fused chunk its
// partial sums plus a read-only pass over the parity-0 sites, else a pass
// over each parity
lgf_status measure_fixed_field(lgf_lattice *h, int format, const void *links, const void *gf, bool fused,
                               double *F, double *theta)
{
    int n0 = 0, n1 = 0;
    if (fused) {
        const int ng = (int)lgf::fixed_sweep_groups(h->geom, h->tune_fixed[format]);
        LGF_HIP(lgf::launch_measure_fixed(format, links, gf, h->geom, 0, h->d_fused + 2 * (size_t)ng, &n0, h->stream,
                                          fixed_records(h, format)));
        LGF_HIP(lgf::launch_finish_measure(h->d_fused, ng + n0, (double)h->V, h->d_out, h->stream));
    } else {
        // the two passes' partial sums in the fused-measurement buffer
        LGF_TRY(ensure_fused_cap(h, 2 * (size_t)lgf::fixed_measure_blocks(h->geom)));
        LGF_HIP(lgf::launch_measure_fixed(format, links, gf, h->geom, 0, h->d_fused, &n0, h->stream,
                                          fixed_records(h, format)));
        LGF_HIP(lgf::launch_measure_fixed(format, links, gf, h->geom, 1, h->d_fused + 2 * (size_t)n0, &n1,
                                          h->stream, fixed_records(h, format)));
        LGF_HIP(lgf::launch_finish_measure(h->d_fused, n0 + n1, (double)h->V, h->d_out, h->stream));
    }
    LGF_HIP(hipMemcpyAsync(h->h_out, h->d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    if (F) *F = h->h_out[0];
    if (theta) *theta = h->h_out[1];
    return LGF_OK;
}

// per-timeslice F_C(t), theta_C(t) of the links g U g^dag into h->h_cout
lgf_status measure_coulomb_fixed_field(lgf_lattice *h, int format, const void *links, const void *gf)
{
    const int bps = lgf::coulomb_fixed_blocks(h->geom);
    const size_t half = (size_t)2 * h->dims[0] * bps;
    const bool rec = fixed_records(h, format);
    LGF_HIP(lgf::launch_measure_coulomb_fixed(format, links, gf, h->geom, 0, h->d_cpart, h->stream, rec));
    LGF_HIP(lgf::launch_measure_coulomb_fixed(format, links, gf, h->geom, 1, h->d_cpart + half, h->stream, rec));
    LGF_HIP(lgf::launch_finish_coulomb(h->d_cpart, h->geom, bps, h->d_cout, h->stream));
    LGF_HIP(hipMemcpyAsync(h->h_cout, h->d_cout, 2 * h->dims[0] * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    return LGF_OK;
}

// lgf_gauge_fix with fixed_links set (the parameters are checked by the
// caller): the same chunks, measurements and precision switch, on (U, g)
// instead of on the links; at the end the handle's links become
// g(x) U_mu(x) g(x+mu)^dag, computed from the untouched input.
lgf_status gauge_fix_fixed(lgf_lattice *h, const lgf_fix_params &p, int bulk, int finish, lgf_fix_result *res,
                           double *history, int history_cap)
{
    const bool mixed = (bulk != finish);
    const auto t_start = std::chrono::steady_clock::now();
    int nh = 0;
    auto record = [&](int64_t sweeps, double F, double th) {
        if (history && nh < history_cap) {
            history[3 * nh] = (double)sweeps;
            history[3 * nh + 1] = F;
            history[3 * nh + 2] = th;
            ++nh;
        }
    };
    auto timed = [&](double &acc_ms, auto &&body) -> lgf_status {
        LGF_HIP(hipEventRecord(h->ev0, h->stream));
        LGF_TRY(body());
        LGF_HIP(hipEventRecord(h->ev1, h->stream));
        LGF_HIP(hipEventSynchronize(h->ev1));
        acc_ms += elapsed_ms(h->ev0, h->ev1);
        return LGF_OK;
    };

    double F = 0.0, theta = 0.0;
    LGF_TRY(timed(res->t_measure_ms, [&]() { return measure_field(h, h->format, h->field, false, &F, &theta); }));
    record(0, F, theta);

    int64_t sweeps = 0, sweeps_bulk = 0;
    uint64_t ctr = p.sweep_offset;
    lgf_status status = LGF_ENOTCONV;
    if (!std::isfinite(F) || !std::isfinite(theta)) status = LGF_ENUMERIC;
    else if (theta < p.theta_target) status = LGF_OK;

    bool in_bulk = mixed;
    int cur = in_bulk ? bulk : finish;
    void *links = nullptr;
    bool started = false;
    if (status == LGF_ENOTCONV && p.max_sweeps > 0) {
        LGF_TRY(ensure_gfix(h, cur));
        LGF_TRY(timed(res->t_convert_ms, [&]() -> lgf_status {
            LGF_TRY(fixed_links(h, cur, &links));
            LGF_HIP(lgf::launch_site_field(gf_format(cur), gfix_of(h, cur), h->geom, 0, h->stream));
            return LGF_OK;
        }));
        started = true;
    }
    const bool fuse = !p.separate_measure;
    for (;;) {
        while (status == LGF_ENOTCONV && sweeps < p.max_sweeps) {
            const int64_t left = p.max_sweeps - sweeps;
            const int n = (int)(left < p.check_every ? left : p.check_every);
            LGF_TRY(timed(in_bulk ? res->t_sweep_bulk_ms : res->t_sweep_finish_ms, [&]() {
                return run_chunk_fixed(h, cur, links, gfix_of(h, cur), n, p.omega, p.p_sr, p.seed, ctr,
                                       p.use_graph != 0, fuse);
            }));
            if (in_bulk) sweeps_bulk += n;
            sweeps += n;
            ctr += (uint64_t)n;
            LGF_TRY(timed(res->t_measure_ms,
                          [&]() { return measure_fixed_field(h, cur, links, gfix_of(h, cur), fuse, &F, &theta); }));
            record(sweeps, F, theta);
            if (!std::isfinite(F) || !std::isfinite(theta)) {
                status = LGF_ENUMERIC;
                break;
            }
            if (in_bulk && (theta < p.theta_switch || theta < p.theta_target)) {
                // the finish precision starts from the bulk's g, reunitarized in
                // FP64, on the links of its own format (the input itself when the
                // formats agree)
                LGF_TRY(ensure_gfix(h, finish));
                LGF_TRY(timed(res->t_convert_ms, [&]() -> lgf_status {
                    LGF_TRY(fixed_links(h, finish, &links));
                    // FP64-12 and the split format share one g field (stored
                    // reunitarized by the chunk's last sweep): nothing to hand over
                    if (gf_format(bulk) != gf_format(finish))
                        LGF_HIP(lgf::launch_site_convert(gf_format(bulk), gfix_of(h, bulk), gf_format(finish),
                                                         gfix_of(h, finish), h->geom, h->stream));
                    return LGF_OK;
                }));
                cur = finish;
                in_bulk = false;
                if (theta < p.theta_target) {
                    LGF_TRY(timed(res->t_measure_ms, [&]() {
                        return measure_fixed_field(h, cur, links, gfix_of(h, cur), false, &F, &theta);
                    }));
                    record(sweeps, F, theta);
                } else {
                    continue;
                }
            }
            if (!in_bulk && theta < p.theta_target) status = LGF_OK;
        }
        if (started) {
            // the links in the final gauge, from the untouched input (element-wise
            // per link, so in place)
            LGF_TRY(timed(res->t_convert_ms, [&]() -> lgf_status {
                LGF_HIP(lgf::launch_gauge_transform(h->format, h->field, gf_format(cur), gfix_of(h, cur), h->format,
                                                    h->field, h->geom, h->stream));
                return LGF_OK;
            }));
            if (cur == LGF_FP64_12S) {
                // the sweeps measured on the split links (within 2^-40 of the
                // input's): F and theta of the result from the FP64 links themselves
                LGF_TRY(timed(res->t_measure_ms,
                              [&]() { return measure_field(h, h->format, h->field, false, &F, &theta); }));
                record(sweeps, F, theta);
                if (!std::isfinite(F) || !std::isfinite(theta)) {
                    status = LGF_ENUMERIC;
                } else if (status == LGF_OK && !(theta < p.theta_target)) {
                    // the split links' fixed point is not yet below the target on
                    // the FP64 links: go on in FP64-12 from the transformed links,
                    // g starting again at 1, while max_sweeps allows
                    status = LGF_ENOTCONV;
                    if (sweeps < p.max_sweeps) {
                        LGF_TRY(ensure_gfix(h, LGF_FP64_12));
                        LGF_TRY(timed(res->t_convert_ms, [&]() -> lgf_status {
                            LGF_TRY(fixed_links(h, LGF_FP64_12, &links));
                            LGF_HIP(lgf::launch_site_field(LGF_FP64_12, gfix_of(h, LGF_FP64_12), h->geom, 0,
                                                           h->stream));
                            return LGF_OK;
                        }));
                        cur = LGF_FP64_12;
                        continue;
                    }
                }
            }
        }
        break;
    }
    res->sweeps = sweeps;
    res->sweeps_bulk = sweeps_bulk;
    res->theta = theta;
    res->F = F;
    res->status = status;
    res->n_history = nh;
    res->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (status == LGF_ENOTCONV)
        return fail(LGF_ENOTCONV, "theta %g after %lld sweeps has not reached %g", theta, (long long)sweeps,
                    p.theta_target);
    if (status == LGF_ENUMERIC) return fail(LGF_ENUMERIC, "F or theta is not finite (F=%g theta=%g)", F, theta);
    return LGF_OK;
}

// lgf_coulomb_gauge_fix with fixed_links set (parameters checked by the
// caller): the per-timeslice stopping and the precision switch of the link
// form, on (U, g); the temporal links are read only by the final
// transformation, which rebuilds all links from the untouched input.
lgf_status coulomb_fix_fixed(lgf_lattice *h, const lgf_fix_params &p, int bulk, int finish, lgf_fix_result *res,
                             double *sweeps_t, double *F_t, double *theta_t)
{
    LGF_TRY(ensure_coulomb(h));
    const int Lt = h->dims[0];
    const bool mixed = (bulk != finish);
    const auto t_start = std::chrono::steady_clock::now();
    std::vector<double> sw(Lt, 0.0), F(Lt), th(Lt);
    std::vector<unsigned char> act(Lt, 1);
    auto timed = [&](double &acc_ms, auto &&body) -> lgf_status {
        LGF_HIP(hipEventRecord(h->ev0, h->stream));
        LGF_TRY(body());
        LGF_HIP(hipEventRecord(h->ev1, h->stream));
        LGF_HIP(hipEventSynchronize(h->ev1));
        acc_ms += elapsed_ms(h->ev0, h->ev1);
        return LGF_OK;
    };
    auto read_out = [&](bool only_active) {
        for (int t = 0; t < Lt; ++t)
            if (!only_active || act[t]) {
                F[t] = h->h_cout[2 * t];
                th[t] = h->h_cout[2 * t + 1];
            }
    };
    auto n_live = [&] {
        int n = 0;
        for (int t = 0; t < Lt; ++t) n += act[t];
        return n;
    };
    auto worst = [&] {
        double m = 0.0;
        for (int t = 0; t < Lt; ++t)
            if (act[t] && th[t] > m) m = th[t];
        return m;
    };
    // the input itself (g = 1)
    LGF_TRY(timed(res->t_measure_ms, [&]() { return measure_coulomb_field(h, h->format, h->field, false); }));
    read_out(false);
    lgf_status status = LGF_ENOTCONV;
    for (int t = 0; t < Lt; ++t) {
        if (!std::isfinite(F[t]) || !std::isfinite(th[t])) status = LGF_ENUMERIC;
        if (th[t] < p.theta_target) act[t] = 0;
    }
    int nh = 1;
    bool in_bulk = mixed, started = false;
    int cur = in_bulk ? bulk : finish;
    void *links = nullptr;
    int64_t sweeps = 0, sweeps_bulk = 0;
    uint64_t ctr = p.sweep_offset;
    if (status != LGF_ENUMERIC && n_live() > 0 && p.max_sweeps > 0) {
        LGF_TRY(ensure_gfix(h, cur));
        LGF_TRY(timed(res->t_convert_ms, [&]() -> lgf_status {
            LGF_TRY(fixed_links(h, cur, &links));
            LGF_HIP(lgf::launch_site_field(gf_format(cur), gfix_of(h, cur), h->geom, 0, h->stream));
            return LGF_OK;
        }));
        started = true;
    }
    while (status != LGF_ENUMERIC && n_live() > 0 && sweeps < p.max_sweeps) {
        LGF_TRY(upload_mask(h, act.data()));
        const int64_t left = p.max_sweeps - sweeps;
        const int n = (int)(left < p.check_every ? left : p.check_every);
        LGF_TRY(timed(in_bulk ? res->t_sweep_bulk_ms : res->t_sweep_finish_ms, [&]() {
            return run_chunk_fixed(h, cur, links, gfix_of(h, cur), n, p.omega, p.p_sr, p.seed, ctr,
                                   p.use_graph != 0, false, true);
        }));
        if (in_bulk) sweeps_bulk += n;
        sweeps += n;
        ctr += (uint64_t)n;
        LGF_TRY(timed(res->t_measure_ms, [&]() { return measure_coulomb_fixed_field(h, cur, links, gfix_of(h, cur)); }));
        read_out(true);
        ++nh;
        for (int t = 0; t < Lt; ++t) {
            if (!act[t]) continue;
            sw[t] = (double)sweeps;
            if (!std::isfinite(F[t]) || !std::isfinite(th[t])) status = LGF_ENUMERIC;
        }
        if (status == LGF_ENUMERIC) break;
        if (in_bulk) {
            // leave the bulk precision once every live timeslice is below the switch
            if (worst() < p.theta_switch) {
                LGF_TRY(ensure_gfix(h, finish));
                LGF_TRY(timed(res->t_convert_ms, [&]() -> lgf_status {
                    LGF_TRY(fixed_links(h, finish, &links));
                    LGF_HIP(lgf::launch_site_convert(gf_format(bulk), gfix_of(h, bulk), gf_format(finish),
                                                     gfix_of(h, finish), h->geom, h->stream));
                    return LGF_OK;
                }));
                cur = finish;
                in_bulk = false;
            }
            continue;
        }
        for (int t = 0; t < Lt; ++t)
            if (act[t] && th[t] < p.theta_target) act[t] = 0;
    }
    if (status != LGF_ENUMERIC) status = n_live() == 0 ? LGF_OK : LGF_ENOTCONV;
    if (started) {
        LGF_TRY(timed(res->t_convert_ms, [&]() -> lgf_status {
            LGF_HIP(lgf::launch_gauge_transform(h->format, h->field, gf_format(cur), gfix_of(h, cur), h->format,
                                                h->field, h->geom, h->stream));
            return LGF_OK;
        }));
        if (cur == LGF_FP64_12S) {
            // the sweeps measured on the split links: every timeslice's F_C and
            // theta_C of the result from the FP64 links themselves
            LGF_TRY(timed(res->t_measure_ms, [&]() { return measure_coulomb_field(h, h->format, h->field, false); }));
            read_out(false);
            if (status == LGF_OK)
                for (int t = 0; t < Lt; ++t)
                    if (!(th[t] < p.theta_target)) status = LGF_ENOTCONV;
        }
    }
    double tmax = 0.0, fsum = 0.0;
    for (int t = 0; t < Lt; ++t) {
        tmax = th[t] > tmax ? th[t] : tmax;
        fsum += F[t];
        if (sweeps_t) sweeps_t[t] = sw[t];
        if (F_t) F_t[t] = F[t];
        if (theta_t) theta_t[t] = th[t];
    }
    res->sweeps = sweeps;
    res->sweeps_bulk = sweeps_bulk;
    res->theta = tmax;
    res->F = fsum / Lt;
    res->status = status;
    res->n_history = nh;
    res->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (status == LGF_ENOTCONV)
        return fail(LGF_ENOTCONV, "not every timeslice reached theta_C < %g in %lld sweeps", p.theta_target,
                    (long long)sweeps);
    if (status == LGF_ENUMERIC) return fail(LGF_ENUMERIC, "F_C or theta_C is not finite");
    return LGF_OK;
}

}  // namespace

extern "C" {

const char *lgf_last_error(void) { return lgf::last_error(); }

const char *lgf_version(void) { return "lgf-mi355x 0.1 (gfx950)"; }

lgf_status lgf_fix_params_default(lgf_fix_params *p)
{
    if (!p) return fail(LGF_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->omega = 1.7;
    p->p_sr = 0.0;
    p->theta_target = 1e-14;
    p->theta_switch = 0.0;
    p->bulk_format = -1;
    p->check_every = 20;
    p->use_graph = 1;
    p->finish_format = -1;
    p->accumulate_g = 0;
    p->max_sweeps = 100000;
    p->seed = 0;
    p->sweep_offset = 0;
    return LGF_OK;
}

size_t lgf_required_bytes(const int dims[4], int format)
{
    if (!valid_dims(dims) || !valid_format(format)) return 0;
    size_t V = 1;
    for (int d = 0; d < 4; ++d) V *= (size_t)dims[d];
    return V * 4 * lgf::link_bytes(format);
}

lgf_status lgf_create(const int dims[4], int format, void *stream, void *device_buf, size_t buf_bytes,
                      lgf_lattice **out)
{
    if (!out) return fail(LGF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dims) return fail(LGF_EINVAL, "dims is NULL");
    if (!valid_dims(dims))
        return fail(LGF_EINVAL, "dims {%d,%d,%d,%d}: every extent must be even and >= 2, V <= 2^31",
                    dims[0], dims[1], dims[2], dims[3]);
    if (!valid_format(format)) return fail(LGF_EINVAL, "unknown format %d", format);
    const size_t need = lgf_required_bytes(dims, format);
    if (device_buf && buf_bytes < need)
        return fail(LGF_EINVAL, "borrowed buffer has %zu bytes, the field needs %zu", buf_bytes, need);

    lgf_lattice *h = new (std::nothrow) lgf_lattice();
    if (!h) return fail(LGF_ENOMEM, "host allocation of the handle failed");
    for (int d = 0; d < 4; ++d) h->dims[d] = dims[d];
    h->V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    h->geom = make_geom(dims);
    h->format = format;
    h->field_bytes = need;
    // defaults: one lane per site, 128-thread workgroups, non-temporal
    // streaming (fastest measured at 64^4 for every format)
    for (int f = 0; f < 4; ++f) h->tune[f] = default_tuning(f);
    for (int f = 0; f <= LGF_FP64_12S; ++f) h->tune_fixed[f] = default_fixed_tuning(f, h->V);

    auto bail = [&](lgf_status st) {
        lgf_destroy(h);
        return st;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return bail(fail(LGF_EHIP, "hipGetDevice: %s", hipGetErrorString(e)));
    if (stream) {
        h->stream = (hipStream_t)stream;
        h->own_stream = false;
    } else {
        e = hipStreamCreate(&h->stream);
        if (e != hipSuccess) return bail(fail(LGF_EHIP, "hipStreamCreate: %s", hipGetErrorString(e)));
        h->own_stream = true;
    }
    if (device_buf) {
        h->field = device_buf;
        h->owned = false;
    } else {
        e = hipMalloc(&h->field, need);
        if (e != hipSuccess) {
            h->field = nullptr;
            (void)hipGetLastError();
            return bail(fail(LGF_ENOMEM, "cannot allocate %zu bytes for the link field", need));
        }
        h->owned = true;
    }
    const int nb = lgf::measure_blocks(h->geom);
    if ((e = hipMalloc(&h->d_partials, (size_t)4 * nb * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&h->d_out, 2 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&h->d_sweep_base, sizeof(uint64_t))) != hipSuccess ||
        (e = hipHostMalloc((void **)&h->h_out, 2 * sizeof(double), hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreate(&h->ev0)) != hipSuccess || (e = hipEventCreate(&h->ev1)) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(LGF_ENOMEM, "handle scratch allocation failed: %s", hipGetErrorString(e)));
    }
    *out = h;
    return LGF_OK;
}

lgf_status lgf_destroy(lgf_lattice *h)
{
    if (!h) return LGF_OK;
    (void)use_device(h);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->owned && h->field) (void)hipFree(h->field);
    for (int f = 0; f < 4; ++f) {
        if (h->work[f]) (void)hipFree(h->work[f]);
        if (h->partner[f]) (void)hipFree(h->partner[f]);
        if (h->gfix[f]) (void)hipFree(h->gfix[f]);
    }
    if (h->split) (void)hipFree(h->split);
    for (int f = 0; f < 5; ++f)
        if (h->rec[f]) (void)hipFree(h->rec[f]);
    if (h->d_partials) (void)hipFree(h->d_partials);
    if (h->d_fused) (void)hipFree(h->d_fused);
    if (h->d_sweep_base) (void)hipFree(h->d_sweep_base);
    if (h->d_trials) (void)hipFree(h->d_trials);
    if (h->d_out) (void)hipFree(h->d_out);
    if (h->h_out) (void)hipHostFree(h->h_out);
    if (h->d_stage) (void)hipFree(h->d_stage);
    if (h->d_sites) (void)hipFree(h->d_sites);
    if (h->d_mask) (void)hipFree(h->d_mask);
    if (h->gacc) (void)hipFree(h->gacc);
    if (h->h_mask) (void)hipHostFree(h->h_mask);
    if (h->d_cpart) (void)hipFree(h->d_cpart);
    if (h->d_cout) (void)hipFree(h->d_cout);
    if (h->h_cout) (void)hipHostFree(h->h_cout);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return LGF_OK;
}

lgf_status lgf_get_info(const lgf_lattice *h, int dims[4], int *format)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    if (dims)
        for (int d = 0; d < 4; ++d) dims[d] = h->dims[d];
    if (format) *format = h->format;
    return LGF_OK;
}

lgf_status lgf_load_links(lgf_lattice *h, const double *host_canon, size_t n_doubles)
{
    if (!h || !host_canon) return fail(LGF_EINVAL, "NULL handle or host array");
    h->fix_on = false;
    if (n_doubles != (size_t)h->V * 72)
        return fail(LGF_EINVAL, "host array has %zu doubles, the lattice needs %lld", n_doubles,
                    (long long)h->V * 72);
    LGF_TRY(use_device(h));
    LGF_TRY(ensure_stage(h));
    for (int64_t s0 = 0; s0 < h->V; s0 += kStageSites) {
        const int64_t n = (h->V - s0 < kStageSites) ? h->V - s0 : kStageSites;
        LGF_HIP(hipMemcpyAsync(h->d_stage, host_canon + s0 * 72, (size_t)n * 72 * sizeof(double),
                               hipMemcpyHostToDevice, h->stream));
        LGF_HIP(lgf::launch_canon_to_field(h->format, h->d_stage, s0, n, h->field, h->geom, h->stream));
    }
    LGF_HIP(hipStreamSynchronize(h->stream));
    return LGF_OK;
}

lgf_status lgf_store_links(lgf_lattice *h, double *host_canon, size_t n_doubles)
{
    if (!h || !host_canon) return fail(LGF_EINVAL, "NULL handle or host array");
    if (n_doubles != (size_t)h->V * 72)
        return fail(LGF_EINVAL, "host array has %zu doubles, the lattice needs %lld", n_doubles,
                    (long long)h->V * 72);
    LGF_TRY(use_device(h));
    LGF_TRY(ensure_stage(h));
    for (int64_t s0 = 0; s0 < h->V; s0 += kStageSites) {
        const int64_t n = (h->V - s0 < kStageSites) ? h->V - s0 : kStageSites;
        LGF_HIP(lgf::launch_field_to_canon(h->format, h->field, nullptr, s0, n, h->d_stage, h->geom,
                                           h->stream));
        LGF_HIP(hipMemcpyAsync(host_canon + s0 * 72, h->d_stage, (size_t)n * 72 * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
        LGF_HIP(hipStreamSynchronize(h->stream));
    }
    return LGF_OK;
}

lgf_status lgf_peek_links(lgf_lattice *h, const int64_t *sites, int64_t n_sites, double *host_out)
{
    if (!h || !sites || !host_out) return fail(LGF_EINVAL, "NULL handle, site list or output");
    if (n_sites < 0) return fail(LGF_EINVAL, "negative site count");
    if (n_sites == 0) return LGF_OK;
    for (int64_t i = 0; i < n_sites; ++i)
        if (sites[i] < 0 || sites[i] >= h->V)
            return fail(LGF_EINVAL, "site %lld is outside [0, %lld)", (long long)sites[i], (long long)h->V);
    LGF_TRY(use_device(h));
    LGF_TRY(ensure_stage(h));
    for (int64_t i0 = 0; i0 < n_sites; i0 += kStageSites) {
        const int64_t n = (n_sites - i0 < kStageSites) ? n_sites - i0 : kStageSites;
        LGF_TRY(ensure_sites(h, n));
        LGF_HIP(hipMemcpyAsync(h->d_sites, sites + i0, (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice,
                               h->stream));
        LGF_HIP(lgf::launch_field_to_canon(h->format, h->field, h->d_sites, 0, n, h->d_stage, h->geom,
                                           h->stream));
        LGF_HIP(hipMemcpyAsync(host_out + i0 * 72, h->d_stage, (size_t)n * 72 * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
        LGF_HIP(hipStreamSynchronize(h->stream));
    }
    return LGF_OK;
}

lgf_status lgf_generate_links(lgf_lattice *h, uint64_t seed, double eps, int haar)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(LGF_EINVAL, "eps must be finite and >= 0");
    LGF_TRY(use_device(h));
    LGF_HIP(lgf::launch_generate(h->format, h->field, h->geom, seed, eps, haar != 0, h->stream));
    return LGF_OK;
}

lgf_status lgf_convert(lgf_lattice *h, int format)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    if (!valid_format(format)) return fail(LGF_EINVAL, "unknown format %d", format);
    if (format == h->format) return LGF_OK;
    if (!h->owned) return fail(LGF_ESTATE, "cannot change the format of a borrowed buffer");
    LGF_TRY(use_device(h));
    const size_t bytes = (size_t)h->V * 4 * lgf::link_bytes(format);
    void *nf = nullptr;
    if (hipMalloc(&nf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LGF_ENOMEM, "cannot allocate %zu bytes for the converted field", bytes);
    }
    const bool to_fp64 = (format == LGF_FP64_18 || format == LGF_FP64_12);
    hipError_t e = lgf::launch_convert(h->format, h->field, format, nf, h->geom, to_fp64, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        (void)hipFree(nf);
        return fail(LGF_EHIP, "format conversion: %s", hipGetErrorString(e));
    }
    drop_graphs(h);
    (void)hipFree(h->field);
    h->field = nf;
    h->field_bytes = bytes;
    h->format = format;
    return LGF_OK;
}

lgf_status lgf_sweep(lgf_lattice *h, int parity, double omega, double p_sr, uint64_t seed,
                     uint64_t sweep_index)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    if (parity < 0 || parity > 2) return fail(LGF_EINVAL, "parity must be 0, 1 or 2 (both)");
    if (!(omega >= 1.0 && omega <= 2.0)) return fail(LGF_EINVAL, "omega %g outside [1, 2]", omega);
    if (!(p_sr >= 0.0 && p_sr <= 1.0)) return fail(LGF_EINVAL, "p_sr %g outside [0, 1]", p_sr);
    LGF_TRY(use_device(h));
    if (parity == 2) {
        prepare_schedule(h, h->format);
        LGF_TRY(full_sweep(h, h->format, h->field, omega, p_sr, seed, sweep_index));
    } else {
        LGF_TRY(sweep_launch(h, h->format, h->field, parity, omega, p_sr, seed, sweep_index));
    }
    return LGF_OK;
}

lgf_status lgf_reunitarize(lgf_lattice *h)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    LGF_TRY(use_device(h));
    LGF_HIP(lgf::launch_convert(h->format, h->field, h->format, h->field, h->geom, true, h->stream));
    return LGF_OK;
}

lgf_status lgf_measure(lgf_lattice *h, double *F, double *theta)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    LGF_TRY(use_device(h));
    return measure_field(h, h->format, h->field, false, F, theta);
}

lgf_status lgf_synchronize(lgf_lattice *h)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    LGF_TRY(use_device(h));
    LGF_HIP(hipStreamSynchronize(h->stream));
    return LGF_OK;
}

lgf_status lgf_gauge_fix(lgf_lattice *h, const lgf_fix_params *pp, lgf_fix_result *res, double *history,
                         int history_cap)
{
    if (!h || !pp || !res) return fail(LGF_EINVAL, "NULL handle, params or result");
    h->fix_on = false;
    const lgf_fix_params p = *pp;
    if (!(p.omega >= 1.0 && p.omega <= 2.0)) return fail(LGF_EINVAL, "omega %g outside [1, 2]", p.omega);
    if (!(p.p_sr >= 0.0 && p.p_sr <= 1.0)) return fail(LGF_EINVAL, "p_sr %g outside [0, 1]", p.p_sr);
    if (!(p.theta_target > 0.0)) return fail(LGF_EINVAL, "theta_target must be > 0");
    if (p.check_every < 1) return fail(LGF_EINVAL, "check_every must be >= 1");
    if (p.max_sweeps < 0) return fail(LGF_EINVAL, "max_sweeps must be >= 0");
    if (history_cap < 0 || (history_cap > 0 && !history)) return fail(LGF_EINVAL, "bad history buffer");
    const int bulk = (p.bulk_format < 0) ? h->format : p.bulk_format;
    const int finish = (p.finish_format < 0) ? h->format : p.finish_format;
    // LGF_FP64_12S: the fixed-link form's sweeps only
    auto valid = [&](int f) { return p.fixed_links ? valid_fixed_format(f) : valid_format(f); };
    if (!valid(bulk)) return fail(LGF_EINVAL, "unknown bulk format %d", bulk);
    if (!valid(finish)) return fail(LGF_EINVAL, "unknown finish format %d", finish);
    const bool mixed = (bulk != finish);
    if (mixed && !(p.theta_switch > 0.0))
        return fail(LGF_EINVAL, "a bulk format other than the finish format needs theta_switch > 0");
    auto is64 = [](int f) { return f == LGF_FP64_18 || f == LGF_FP64_12; };
    const bool acc = p.accumulate_g != 0;
    // the sweeps accumulate into g only inside this call, whatever way it ends
    struct AccOff {
        lgf_lattice *h;
        ~AccOff() { h->gacc_active = nullptr; }
    } acc_off{h};
    if (p.fixed_links) {
        if (!is64(h->format)) return fail(LGF_EINVAL, "fixed_links needs an FP64 handle");
        LGF_TRY(use_device(h));
        std::memset(res, 0, sizeof *res);
        return gauge_fix_fixed(h, p, bulk, finish, res, history, history_cap);
    }
    if (acc && !(mixed && !is64(bulk) && is64(finish) && is64(h->format)))
        return fail(LGF_EINVAL, "accumulate_g needs an FP32 bulk, an FP64 finish and an FP64 handle");
    LGF_TRY(use_device(h));

    std::memset(res, 0, sizeof *res);
    const auto t_start = std::chrono::steady_clock::now();
    int nh = 0;
    auto record = [&](int64_t sweeps, double F, double th) {
        if (history && nh < history_cap) {
            history[3 * nh] = (double)sweeps;
            history[3 * nh + 1] = F;
            history[3 * nh + 2] = th;
            ++nh;
        }
    };
    // the field the sweeps run on, and a timed conversion between fields
    int cur_fmt = h->format;
    void *cur = h->field;
    auto move_to = [&](int fmt, bool reunit) -> lgf_status {
        void *dst = h->field;
        if (fmt != h->format) {
            LGF_TRY(ensure_work(h, fmt));
            dst = h->work[fmt];
        }
        if (dst == cur) return LGF_OK;
        LGF_HIP(hipEventRecord(h->ev0, h->stream));
        LGF_HIP(lgf::launch_convert(cur_fmt, cur, fmt, dst, h->geom, reunit, h->stream));
        LGF_HIP(hipEventRecord(h->ev1, h->stream));
        LGF_HIP(hipEventSynchronize(h->ev1));
        res->t_convert_ms += elapsed_ms(h->ev0, h->ev1);
        cur = dst;
        cur_fmt = fmt;
        return LGF_OK;
    };
    auto measure_timed = [&](bool reunit, double *F, double *th) -> lgf_status {
        LGF_HIP(hipEventRecord(h->ev0, h->stream));
        LGF_TRY(measure_field(h, cur_fmt, cur, reunit, F, th));
        LGF_HIP(hipEventRecord(h->ev1, h->stream));
        LGF_HIP(hipEventSynchronize(h->ev1));
        res->t_measure_ms += elapsed_ms(h->ev0, h->ev1);
        return LGF_OK;
    };

    double F = 0.0, theta = 0.0;
    LGF_TRY(measure_timed(false, &F, &theta));
    record(0, F, theta);

    int64_t sweeps = 0, sweeps_bulk = 0;
    uint64_t ctr = p.sweep_offset;
    lgf_status status = LGF_ENOTCONV;
    if (!std::isfinite(F) || !std::isfinite(theta)) status = LGF_ENUMERIC;
    else if (theta < p.theta_target) status = LGF_OK;

    bool in_bulk = mixed;
    if (status == LGF_ENOTCONV && p.max_sweeps > 0) {
        const int first = in_bulk ? bulk : finish;
        const bool to_fp64 = (first == LGF_FP64_18 || first == LGF_FP64_12) &&
                             !(h->format == LGF_FP64_18 || h->format == LGF_FP64_12);
        LGF_TRY(move_to(first, to_fp64));
        if (acc && in_bulk) LGF_TRY(gacc_begin(h, bulk));
    }
    while (status == LGF_ENOTCONV && sweeps < p.max_sweeps) {
        const int64_t left = p.max_sweeps - sweeps;
        const int n = (int)(left < p.check_every ? left : p.check_every);
        // reunitarize + measure inside the chunk's last half-sweep where possible
        const bool fuse = !p.separate_measure && can_fuse(h, cur_fmt, p.p_sr, false);
        LGF_HIP(hipEventRecord(h->ev0, h->stream));
        LGF_TRY(run_chunk(h, cur_fmt, cur, n, p.omega, p.p_sr, p.seed, ctr, p.use_graph != 0, false, fuse));
        LGF_HIP(hipEventRecord(h->ev1, h->stream));
        LGF_HIP(hipEventSynchronize(h->ev1));
        const double ms = elapsed_ms(h->ev0, h->ev1);
        if (in_bulk) {
            res->t_sweep_bulk_ms += ms;
            sweeps_bulk += n;
        } else {
            res->t_sweep_finish_ms += ms;
        }
        sweeps += n;
        ctr += (uint64_t)n;

        if (h->gacc_active) LGF_HIP(lgf::launch_site_field(bulk, h->gacc, h->geom, 1, h->stream));
        if (fuse) {
            LGF_HIP(hipEventRecord(h->ev0, h->stream));
            LGF_TRY(measure_fused(h, cur_fmt, cur, &F, &theta));
            LGF_HIP(hipEventRecord(h->ev1, h->stream));
            LGF_HIP(hipEventSynchronize(h->ev1));
            res->t_measure_ms += elapsed_ms(h->ev0, h->ev1);
        } else {
            LGF_TRY(measure_timed(true, &F, &theta));
        }
        record(sweeps, F, theta);
        if (!std::isfinite(F) || !std::isfinite(theta)) {
            status = LGF_ENUMERIC;
            break;
        }
        if (in_bulk && (theta < p.theta_switch || theta < p.theta_target)) {
            if (h->gacc_active) {
                // rebuild the FP64 links from the untouched FP64 input: an exact
                // gauge transformation by the accumulated g
                void *dst = h->field;
                if (finish != h->format) {
                    LGF_TRY(ensure_work(h, finish));
                    dst = h->work[finish];
                }
                LGF_HIP(hipEventRecord(h->ev0, h->stream));
                LGF_TRY(gacc_apply(h, bulk, finish, dst));
                LGF_HIP(hipEventRecord(h->ev1, h->stream));
                LGF_HIP(hipEventSynchronize(h->ev1));
                res->t_convert_ms += elapsed_ms(h->ev0, h->ev1);
                cur = dst;
                cur_fmt = finish;
            } else {
                // leave the bulk precision, reunitarizing in FP64 on the way
                LGF_TRY(move_to(finish, true));
            }
            in_bulk = false;
            if (theta < p.theta_target) {
                LGF_TRY(measure_timed(false, &F, &theta));
                record(sweeps, F, theta);
            } else {
                continue;
            }
        }
        if (!in_bulk && theta < p.theta_target) status = LGF_OK;
    }
    if (h->gacc_active) {
        // stopped inside the bulk (max_sweeps): hand back the exact transform
        LGF_TRY(gacc_apply(h, bulk, h->format, h->field));
        cur = h->field;
        cur_fmt = h->format;
    }
    // hand the links back in the handle's own format
    LGF_TRY(move_to(h->format, false));

    res->sweeps = sweeps;
    res->sweeps_bulk = sweeps_bulk;
    res->theta = theta;
    res->F = F;
    res->status = status;
    res->n_history = nh;
    res->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (status == LGF_ENOTCONV)
        return fail(LGF_ENOTCONV, "theta %g after %lld sweeps has not reached %g", theta, (long long)sweeps,
                    p.theta_target);
    if (status == LGF_ENUMERIC) return fail(LGF_ENUMERIC, "F or theta is not finite (F=%g theta=%g)", F, theta);
    return LGF_OK;
}

lgf_status lgf_fix_begin(lgf_lattice *h, int format)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    if (!valid_fixed_format(format)) return fail(LGF_EINVAL, "unknown format %d", format);
    if (h->format != LGF_FP64_18 && h->format != LGF_FP64_12)
        return fail(LGF_EINVAL, "the fixed-link form needs an FP64 handle");
    LGF_TRY(use_device(h));
    void *links = nullptr;
    LGF_TRY(ensure_gfix(h, format));
    LGF_TRY(fixed_links(h, format, &links));
    LGF_HIP(lgf::launch_site_field(gf_format(format), gfix_of(h, format), h->geom, 0, h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    h->fix_format = format;
    h->fix_links = links;
    h->fix_on = true;
    return LGF_OK;
}

lgf_status lgf_fix_chunk(lgf_lattice *h, int n, double omega, double p_sr, uint64_t seed, uint64_t sweep0,
                         int use_graph, double *F, double *theta, double *sweep_ms)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    if (!h->fix_on) return fail(LGF_ESTATE, "no stepwise gauge fixing open (lgf_fix_begin)");
    if (n < 1) return fail(LGF_EINVAL, "n must be >= 1");
    if (!(omega >= 1.0 && omega <= 2.0)) return fail(LGF_EINVAL, "omega %g outside [1, 2]", omega);
    if (!(p_sr >= 0.0 && p_sr <= 1.0)) return fail(LGF_EINVAL, "p_sr %g outside [0, 1]", p_sr);
    LGF_TRY(use_device(h));
    const int fmt = h->fix_format;
    void *gf = gfix_of(h, fmt);
    LGF_HIP(hipEventRecord(h->ev0, h->stream));
    LGF_TRY(run_chunk_fixed(h, fmt, h->fix_links, gf, n, omega, p_sr, seed, sweep0, use_graph != 0, true));
    LGF_HIP(hipEventRecord(h->ev1, h->stream));
    double f = 0.0, th = 0.0;
    LGF_TRY(measure_fixed_field(h, fmt, h->fix_links, gf, true, &f, &th));
    if (sweep_ms) *sweep_ms = elapsed_ms(h->ev0, h->ev1);
    if (F) *F = f;
    if (theta) *theta = th;
    if (!std::isfinite(f) || !std::isfinite(th))
        return fail(LGF_ENUMERIC, "F or theta is not finite (F=%g theta=%g)", f, th);
    return LGF_OK;
}

lgf_status lgf_fix_end(lgf_lattice *h)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    if (!h->fix_on) return fail(LGF_ESTATE, "no stepwise gauge fixing open (lgf_fix_begin)");
    h->fix_on = false;
    LGF_TRY(use_device(h));
    LGF_HIP(lgf::launch_gauge_transform(h->format, h->field, gf_format(h->fix_format), gfix_of(h, h->fix_format),
                                        h->format, h->field, h->geom, h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    return LGF_OK;
}

namespace {

// checks shared by the annealing entry points; allocates the trial counter
lgf_status anneal_ready(lgf_lattice *h)
{
    if (h->format != LGF_FP64_18 && h->format != LGF_FP64_12)
        return fail(LGF_EINVAL, "simulated annealing needs an FP64 handle");
    LGF_TRY(use_device(h));
    if (!h->d_trials) {
        if (hipMalloc(&h->d_trials, sizeof(unsigned long long)) != hipSuccess) {
            h->d_trials = nullptr;
            (void)hipGetLastError();
            return fail(LGF_ENOMEM, "cannot allocate the trial counter");
        }
    }
    return LGF_OK;
}

// the trial counter, read back (synchronises the stream)
lgf_status read_trials(lgf_lattice *h, uint64_t *trials)
{
    LGF_HIP(hipMemcpyAsync(h->h_out, h->d_trials, sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    unsigned long long v;
    std::memcpy(&v, h->h_out, sizeof v);
    *trials = (uint64_t)v;
    return LGF_OK;
}

// temperature of annealing sweep n of n_sweeps, linear from T_start to T_end
// (both ends exact)
double anneal_temperature(int64_t n, int64_t n_sweeps, double T_start, double T_end)
{
#pragma clang fp contract(off)
    if (n_sweeps <= 1) return T_start;
    const double f = (double)n / (double)(n_sweeps - 1);
    return T_start * (1.0 - f) + T_end * f;
}

}  // namespace

lgf_status lgf_anneal_sweep(lgf_lattice *h, int parity, double T, uint64_t seed, uint64_t sweep_index,
                            uint64_t *trials)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    if (parity < 0 || parity > 2) return fail(LGF_EINVAL, "parity must be 0, 1 or 2 (both)");
    if (!(T > 0.0) || !std::isfinite(T)) return fail(LGF_EINVAL, "temperature %g must be finite and > 0", T);
    LGF_TRY(anneal_ready(h));
    unsigned long long *ctr = trials ? h->d_trials : nullptr;
    if (ctr) LGF_HIP(lgf::launch_set_u64(reinterpret_cast<uint64_t *>(ctr), 0, h->stream));
    for (int p = 0; p < 2; ++p)
        if (parity == 2 || parity == p)
            LGF_HIP(lgf::launch_anneal(h->format, h->field, h->geom, p, T, seed, sweep_index, 0u, ctr, h->stream));
    if (trials) LGF_TRY(read_trials(h, trials));
    return LGF_OK;
}

lgf_status lgf_anneal(lgf_lattice *h, int64_t n_sweeps, double T_start, double T_end, uint64_t seed,
                      uint64_t sweep0, uint64_t *trials, double *ms)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    if (n_sweeps < 1) return fail(LGF_EINVAL, "n_sweeps must be >= 1");
    if (!(T_start > 0.0) || !std::isfinite(T_start) || !(T_end > 0.0) || !std::isfinite(T_end))
        return fail(LGF_EINVAL, "temperatures must be finite and > 0 (%g, %g)", T_start, T_end);
    LGF_TRY(anneal_ready(h));
    LGF_HIP(lgf::launch_set_u64(reinterpret_cast<uint64_t *>(h->d_trials), 0, h->stream));
    LGF_HIP(hipEventRecord(h->ev0, h->stream));
    for (int64_t n = 0; n < n_sweeps; ++n) {
        const double T = anneal_temperature(n, n_sweeps, T_start, T_end);
        for (int p = 0; p < 2; ++p)
            LGF_HIP(lgf::launch_anneal(h->format, h->field, h->geom, p, T, seed, sweep0 + (uint64_t)n, 0u,
                                       h->d_trials, h->stream));
        if ((n + 1) % 20 == 0 || n + 1 == n_sweeps)
            LGF_HIP(lgf::launch_convert(h->format, h->field, h->format, h->field, h->geom, true, h->stream));
    }
    LGF_HIP(hipEventRecord(h->ev1, h->stream));
    uint64_t t = 0;
    LGF_TRY(read_trials(h, &t));
    if (trials) *trials = t;
    if (ms) *ms = elapsed_ms(h->ev0, h->ev1);
    return LGF_OK;
}

// ----------------------------------------------------------------------------
// The allocation-free measurement.  Its per-workgroup partial sums live in a
// file-scope device array instead of handle memory; each GPU holds its own
// copy of the array, whose address the runtime gives per device.
// ----------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;  // 4 MiB: (F, theta) partials of up to 2^26 sites
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxScratchDevices];  // device address of `scratch` on each device (set on first use)

// the address of `scratch` on device dev, which must be current
lgf_status scratch_on(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(LGF_EINVAL, "device %d: the scratch table holds devices 0..%d", dev, kMaxScratchDevices - 1);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LGF_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return LGF_OK;
}

}  // namespace

lgf_status lgf_measure_noalloc(lgf_lattice *h, double *d_out)
{
    if (!h || !d_out) return fail(LGF_EINVAL, "NULL handle or output");
    const size_t need = (size_t)4 * (size_t)lgf::measure_blocks(h->geom) * sizeof(double);
    if (need > kScratchBytes)
        return fail(LGF_EINVAL,
                    "a lattice of %lld sites needs %zu bytes of partial sums, more than the %zu bytes of the "
                    "allocation-free measurement (at most 2^26 sites); use lgf_measure",
                    (long long)h->V, need, kScratchBytes);
    LGF_TRY(use_device(h));
    void *scr = nullptr;
    LGF_TRY(scratch_on(h->device, &scr));
    double *part = static_cast<double *>(scr);
    int n0 = 0, n1 = 0;
    LGF_HIP(lgf::launch_measure(h->format, h->field, h->geom, 0, false, false, part, &n0, h->stream));
    LGF_HIP(lgf::launch_measure(h->format, h->field, h->geom, 1, false, false, part + 2 * n0, &n1, h->stream));
    LGF_HIP(lgf::launch_finish_measure(part, n0 + n1, (double)h->V, d_out, h->stream));
    return LGF_OK;
}

lgf_status lgf_plaquette(lgf_lattice *h, double *P)
{
    if (!h || !P) return fail(LGF_EINVAL, "NULL handle or output");
    LGF_TRY(use_device(h));
    int n = 0;
    LGF_HIP(lgf::launch_plaquette(h->format, h->field, h->geom, h->d_partials, &n, h->stream));
    LGF_HIP(lgf::launch_finish_measure(h->d_partials, n, (double)h->V, h->d_out, h->stream));
    LGF_HIP(hipMemcpyAsync(h->h_out, h->d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LGF_HIP(hipStreamSynchronize(h->stream));
    *P = h->h_out[0] * 12.0 / 18.0;  // the final sum divides by 12 V; the plaquette by 18 V
    return LGF_OK;
}

lgf_status lgf_sweep_coulomb(lgf_lattice *h, int parity, double omega, double p_sr, uint64_t seed,
                             uint64_t sweep_index, const unsigned char *slice_active)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    if (parity < 0 || parity > 2) return fail(LGF_EINVAL, "parity must be 0, 1 or 2 (both)");
    if (!(omega >= 1.0 && omega <= 2.0)) return fail(LGF_EINVAL, "omega %g outside [1, 2]", omega);
    if (!(p_sr >= 0.0 && p_sr <= 1.0)) return fail(LGF_EINVAL, "p_sr %g outside [0, 1]", p_sr);
    LGF_TRY(use_device(h));
    LGF_TRY(ensure_coulomb(h));
    LGF_TRY(upload_mask(h, slice_active));
    for (int par = (parity == 1 ? 1 : 0); par <= (parity == 0 ? 0 : 1); ++par)
        LGF_TRY(sweep_launch(h, h->format, h->field, par, omega, p_sr, seed, sweep_index, true));
    return LGF_OK;
}

lgf_status lgf_measure_coulomb(lgf_lattice *h, double *F_t, double *theta_t)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    LGF_TRY(use_device(h));
    LGF_TRY(ensure_coulomb(h));
    LGF_TRY(measure_coulomb_field(h, h->format, h->field, false));
    for (int t = 0; t < h->dims[0]; ++t) {
        if (F_t) F_t[t] = h->h_cout[2 * t];
        if (theta_t) theta_t[t] = h->h_cout[2 * t + 1];
    }
    return LGF_OK;
}

lgf_status lgf_coulomb_gauge_fix(lgf_lattice *h, const lgf_fix_params *pp, lgf_fix_result *res, double *sweeps_t,
                                 double *F_t, double *theta_t)
{
    if (!h || !pp || !res) return fail(LGF_EINVAL, "NULL handle, params or result");
    h->fix_on = false;
    const lgf_fix_params p = *pp;
    if (!(p.omega >= 1.0 && p.omega <= 2.0)) return fail(LGF_EINVAL, "omega %g outside [1, 2]", p.omega);
    if (!(p.p_sr >= 0.0 && p.p_sr <= 1.0)) return fail(LGF_EINVAL, "p_sr %g outside [0, 1]", p.p_sr);
    if (!(p.theta_target > 0.0)) return fail(LGF_EINVAL, "theta_target must be > 0");
    if (p.check_every < 1) return fail(LGF_EINVAL, "check_every must be >= 1");
    if (p.max_sweeps < 0) return fail(LGF_EINVAL, "max_sweeps must be >= 0");
    const int bulk = (p.bulk_format < 0) ? h->format : p.bulk_format;
    const int finish = (p.finish_format < 0) ? h->format : p.finish_format;
    // LGF_FP64_12S: the fixed-link form's sweeps only
    auto valid = [&](int f) { return p.fixed_links ? valid_fixed_format(f) : valid_format(f); };
    if (!valid(bulk) || !valid(finish)) return fail(LGF_EINVAL, "unknown format");
    const bool mixed = bulk != finish;
    if (mixed && !(p.theta_switch > 0.0))
        return fail(LGF_EINVAL, "a bulk format other than the finish format needs theta_switch > 0");
    auto is64 = [](int f) { return f == LGF_FP64_18 || f == LGF_FP64_12; };
    if (p.fixed_links) {
        if (!is64(h->format)) return fail(LGF_EINVAL, "fixed_links needs an FP64 handle");
        LGF_TRY(use_device(h));
        std::memset(res, 0, sizeof *res);
        return coulomb_fix_fixed(h, p, bulk, finish, res, sweeps_t, F_t, theta_t);
    }
    const bool acc = p.accumulate_g != 0;
    if (acc && !(mixed && !is64(bulk) && is64(finish) && is64(h->format)))
        return fail(LGF_EINVAL, "accumulate_g needs an FP32 bulk, an FP64 finish and an FP64 handle");
    // the sweeps accumulate into g only inside this call, whatever way it ends
    struct AccOff {
        lgf_lattice *h;
        ~AccOff() { h->gacc_active = nullptr; }
    } acc_off{h};
    LGF_TRY(use_device(h));
    LGF_TRY(ensure_coulomb(h));
    const int Lt = h->dims[0];
    std::memset(res, 0, sizeof *res);
    const auto t_start = std::chrono::steady_clock::now();
    std::vector<double> sw(Lt, 0.0), F(Lt), th(Lt);
    std::vector<unsigned char> act(Lt, 1);
    int cur_fmt = h->format;
    void *cur = h->field;
    auto move_to = [&](int fmt, bool reunit) -> lgf_status {
        void *dst = h->field;
        if (fmt != h->format) {
            LGF_TRY(ensure_work(h, fmt));
            dst = h->work[fmt];
        }
        if (dst == cur) return LGF_OK;
        LGF_HIP(hipEventRecord(h->ev0, h->stream));
        LGF_HIP(lgf::launch_convert(cur_fmt, cur, fmt, dst, h->geom, reunit, h->stream));
        LGF_HIP(hipEventRecord(h->ev1, h->stream));
        LGF_HIP(hipEventSynchronize(h->ev1));
        res->t_convert_ms += elapsed_ms(h->ev0, h->ev1);
        cur = dst;
        cur_fmt = fmt;
        return LGF_OK;
    };
    auto measure = [&](bool reunit, bool only_active) -> lgf_status {
        LGF_HIP(hipEventRecord(h->ev0, h->stream));
        LGF_TRY(measure_coulomb_field(h, cur_fmt, cur, reunit));
        LGF_HIP(hipEventRecord(h->ev1, h->stream));
        LGF_HIP(hipEventSynchronize(h->ev1));
        res->t_measure_ms += elapsed_ms(h->ev0, h->ev1);
        for (int t = 0; t < Lt; ++t)
            if (!only_active || act[t]) {
                F[t] = h->h_cout[2 * t];
                th[t] = h->h_cout[2 * t + 1];
            }
        return LGF_OK;
    };
    auto n_live = [&] {
        int n = 0;
        for (int t = 0; t < Lt; ++t) n += act[t];
        return n;
    };
    auto worst = [&] {
        double m = 0.0;
        for (int t = 0; t < Lt; ++t)
            if (act[t] && th[t] > m) m = th[t];
        return m;
    };
    lgf_status status = LGF_ENOTCONV;
    LGF_TRY(measure(false, false));
    int nh = 1;
    for (int t = 0; t < Lt; ++t) {
        if (!std::isfinite(F[t]) || !std::isfinite(th[t])) status = LGF_ENUMERIC;
        if (th[t] < p.theta_target) act[t] = 0;
    }
    bool in_bulk = mixed;
    int64_t sweeps = 0, sweeps_bulk = 0;
    uint64_t ctr = p.sweep_offset;
    if (status != LGF_ENUMERIC && n_live() > 0 && p.max_sweeps > 0) {
        const int first = in_bulk ? bulk : finish;
        LGF_TRY(move_to(first, is64(first) && !is64(h->format)));
        if (acc && in_bulk) LGF_TRY(gacc_begin(h, bulk));
    }
    while (status != LGF_ENUMERIC && n_live() > 0 && sweeps < p.max_sweeps) {
        LGF_TRY(upload_mask(h, act.data()));
        const int64_t left = p.max_sweeps - sweeps;
        const int n = (int)(left < p.check_every ? left : p.check_every);
        LGF_HIP(hipEventRecord(h->ev0, h->stream));
        LGF_TRY(run_chunk(h, cur_fmt, cur, n, p.omega, p.p_sr, p.seed, ctr, p.use_graph != 0, true));
        LGF_HIP(hipEventRecord(h->ev1, h->stream));
        LGF_HIP(hipEventSynchronize(h->ev1));
        const double ms = elapsed_ms(h->ev0, h->ev1);
        if (in_bulk) {
            res->t_sweep_bulk_ms += ms;
            sweeps_bulk += n;
        } else {
            res->t_sweep_finish_ms += ms;
        }
        sweeps += n;
        ctr += (uint64_t)n;
        if (h->gacc_active) LGF_HIP(lgf::launch_site_field(bulk, h->gacc, h->geom, 1, h->stream));
        LGF_TRY(measure(true, true));
        ++nh;
        for (int t = 0; t < Lt; ++t) {
            if (!act[t]) continue;
            sw[t] = (double)sweeps;
            if (!std::isfinite(F[t]) || !std::isfinite(th[t])) status = LGF_ENUMERIC;
        }
        if (status == LGF_ENUMERIC) break;
        if (in_bulk) {
            // leave the bulk precision once every live timeslice is below the switch
            if (worst() < p.theta_switch) {
                if (h->gacc_active) {
                    // the FP64 links as an exact gauge transformation of the input
                    void *dst = h->field;
                    if (finish != h->format) {
                        LGF_TRY(ensure_work(h, finish));
                        dst = h->work[finish];
                    }
                    LGF_HIP(hipEventRecord(h->ev0, h->stream));
                    LGF_TRY(gacc_apply(h, bulk, finish, dst));
                    LGF_HIP(hipEventRecord(h->ev1, h->stream));
                    LGF_HIP(hipEventSynchronize(h->ev1));
                    res->t_convert_ms += elapsed_ms(h->ev0, h->ev1);
                    cur = dst;
                    cur_fmt = finish;
                } else {
                    LGF_TRY(move_to(finish, true));
                }
                in_bulk = false;
            }
            continue;
        }
        for (int t = 0; t < Lt; ++t)
            if (act[t] && th[t] < p.theta_target) act[t] = 0;
    }
    if (status != LGF_ENUMERIC) status = n_live() == 0 ? LGF_OK : LGF_ENOTCONV;
    if (h->gacc_active) {
        // stopped inside the bulk: hand back the exact transform of the input
        LGF_TRY(gacc_apply(h, bulk, h->format, h->field));
        cur = h->field;
        cur_fmt = h->format;
    }
    LGF_TRY(move_to(h->format, false));
    double tmax = 0.0, fsum = 0.0;
    for (int t = 0; t < Lt; ++t) {
        tmax = th[t] > tmax ? th[t] : tmax;
        fsum += F[t];
        if (sweeps_t) sweeps_t[t] = sw[t];
        if (F_t) F_t[t] = F[t];
        if (theta_t) theta_t[t] = th[t];
    }
    res->sweeps = sweeps;
    res->sweeps_bulk = sweeps_bulk;
    res->theta = tmax;
    res->F = fsum / Lt;
    res->status = status;
    res->n_history = nh;
    res->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (status == LGF_ENOTCONV)
        return fail(LGF_ENOTCONV, "not every timeslice reached theta_C < %g in %lld sweeps", p.theta_target,
                    (long long)sweeps);
    if (status == LGF_ENUMERIC) return fail(LGF_ENUMERIC, "F_C or theta_C is not finite");
    return LGF_OK;
}

lgf_status lgf_set_tuning(lgf_lattice *h, int format, const lgf_sweep_tuning *t)
{
    if (!h || !t) return fail(LGF_EINVAL, "NULL handle or tuning");
    if (!valid_format(format)) return fail(LGF_EINVAL, "unknown format %d", format);
    const lgf_sweep_tuning u = *t;
    if (u.lanes_per_site != 1 && u.lanes_per_site != 2 && u.lanes_per_site != 4)
        return fail(LGF_EINVAL, "lanes_per_site must be 1, 2 or 4");
    if (u.sites_per_thread != 1 && u.sites_per_thread != 2 && u.sites_per_thread != 4)
        return fail(LGF_EINVAL, "sites_per_thread must be 1, 2 or 4");
    if (u.block != 64 && u.block != 128 && u.block != 256)
        return fail(LGF_EINVAL, "block must be 64, 128 or 256");
    if (u.schedule < lgf::kScheduleInPlace || u.schedule > lgf::kScheduleOutOfPlace)
        return fail(LGF_EINVAL, "schedule must be 0 (in place), 1 (t-slice pipeline) or 2 (out of place)");
    if (u.schedule == lgf::kScheduleOutOfPlace && !u.nontemporal)
        return fail(LGF_EINVAL, "the out-of-place schedule needs nontemporal = 1");
    if (u.schedule == lgf::kScheduleOutOfPlace) {
        LGF_TRY(use_device(h));
        LGF_TRY(ensure_partner(h, format));
    }
    h->tune[format] = lgf::SweepTuning{u.lanes_per_site, u.block,      u.xcd_remap ? 1 : 0, u.nontemporal ? 1 : 0,
                                       u.schedule,       u.sites_per_thread};
    drop_graphs(h);
    return LGF_OK;
}

lgf_status lgf_get_tuning(const lgf_lattice *h, int format, lgf_sweep_tuning *t)
{
    if (!h || !t) return fail(LGF_EINVAL, "NULL handle or tuning");
    if (!valid_format(format)) return fail(LGF_EINVAL, "unknown format %d", format);
    const lgf::SweepTuning &u = h->tune[format];
    t->lanes_per_site = u.lanes_per_site;
    t->sites_per_thread = u.sites_per_thread;
    t->block = u.block;
    t->xcd_remap = u.xcd_remap;
    t->nontemporal = u.nontemporal;
    t->schedule = u.schedule;
    return LGF_OK;
}

lgf_status lgf_set_fixed_tuning(lgf_lattice *h, int format, const lgf_sweep_tuning *t)
{
    if (!h || !t) return fail(LGF_EINVAL, "NULL handle or tuning");
    if (!valid_fixed_format(format)) return fail(LGF_EINVAL, "unknown format %d", format);
    const lgf_sweep_tuning u = *t;
    if (!(u.lanes_per_site == 2 || u.lanes_per_site == 4 ||
          (u.lanes_per_site == 1 && lgf::fixed_one_lane_format(format))))
        return fail(LGF_EINVAL, "the fixed-link sweep takes lanes_per_site 2 or 4 (or 1 in the FP32 formats)");
    if (u.block != 64 && u.block != 128 && u.block != 256) return fail(LGF_EINVAL, "block must be 64, 128 or 256");
    if (u.xcd_remap < 0 || u.xcd_remap > 3) return fail(LGF_EINVAL, "xcd_remap (tile order) must be 0, 1, 2 or 3");
    if (u.sites_per_thread != 1 || u.nontemporal != 1)
        return fail(LGF_EINVAL, "the fixed-link sweep takes sites_per_thread 1, nontemporal 1");
    if (!(u.schedule == lgf::kLayoutPlanes || (u.schedule == lgf::kLayoutRecords && lgf::fixed_records_format(format))))
        return fail(LGF_EINVAL, "schedule (link layout) must be 0, or 1 (per-site records) in FP32-12, FP64-12 and FP64-12S");
    lgf::SweepTuning n{};
    n.lanes_per_site = u.lanes_per_site;
    n.block = u.block;
    n.xcd_remap = u.xcd_remap;
    n.schedule = u.schedule;
    // an open stepwise session holds its links in the layout of the old
    // tuning: it is closed (without applying g)
    h->fix_on = false;
    h->tune_fixed[format] = n;
    drop_graphs(h);
    if (h->rec[format] && n.schedule != lgf::kLayoutRecords) {
        // the link field from now on: the records' memory goes back
        (void)hipFree(h->rec[format]);
        h->rec[format] = nullptr;
    }
    return LGF_OK;
}

lgf_status lgf_get_fixed_tuning(const lgf_lattice *h, int format, lgf_sweep_tuning *t)
{
    if (!h || !t) return fail(LGF_EINVAL, "NULL handle or tuning");
    if (!valid_fixed_format(format)) return fail(LGF_EINVAL, "unknown format %d", format);
    const lgf::SweepTuning &u = h->tune_fixed[format];
    t->lanes_per_site = u.lanes_per_site;
    t->sites_per_thread = u.sites_per_thread;
    t->block = u.block;
    t->xcd_remap = u.xcd_remap;
    t->nontemporal = u.nontemporal;
    t->schedule = u.schedule;
    return LGF_OK;
}

lgf_status lgf_autotune_fixed(lgf_lattice *h, int format, int trials)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    if (!valid_fixed_format(format)) return fail(LGF_EINVAL, "unknown format %d", format);
    if (trials < 1) return fail(LGF_EINVAL, "trials must be >= 1");
    if (h->format != LGF_FP64_18 && h->format != LGF_FP64_12)
        return fail(LGF_EINVAL, "the fixed-link form needs an FP64 handle");
    LGF_TRY(use_device(h));
    // The fixed-link sweeps only read the links (the handle's own, or their
    // working copy in this format, and its per-site records) and write the
    // gauge transformation, which the gauge fixing resets before use: nothing
    // needs saving.
    void *links = nullptr, *records = nullptr;
    LGF_TRY(ensure_gfix(h, format));
    LGF_TRY(links_in_format(h, format, &links));
    if (lgf::fixed_records_format(format)) {
        bool built = false;
        LGF_TRY(build_records(h, format, &built));
        if (built) records = h->rec[format];
    }
    void *gf = gfix_of(h, format);
    LGF_HIP(lgf::launch_site_field(gf_format(format), gf, h->geom, 0, h->stream));
    hipError_t e = hipSuccess;
    auto sweep = [&](const lgf::SweepTuning &t) {
        const void *l = (t.schedule == lgf::kLayoutRecords) ? records : links;
        lgf::SweepArgs a{0, 1.7, 0.0, 0, 0, 0u};
        if (e == hipSuccess) e = lgf::launch_fixed_sweep(format, l, gf, h->geom, a, t, 0, h->stream);
        a.parity = 1;
        if (e == hipSuccess) e = lgf::launch_fixed_sweep(format, l, gf, h->geom, a, t, 0, h->stream);
    };
    auto time_variant = [&](const lgf::SweepTuning &t, int n, double *ms) {
        sweep(t);
        if (e == hipSuccess) e = hipEventRecord(h->ev0, h->stream);
        for (int k = 0; k < n && e == hipSuccess; ++k) sweep(t);
        if (e == hipSuccess) e = hipEventRecord(h->ev1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(h->ev1);
        if (e != hipSuccess) return false;
        *ms = elapsed_ms(h->ev0, h->ev1) / n;
        return true;
    };
    lgf::SweepTuning dflt = default_fixed_tuning(format, h->V);
    if (!records) dflt.schedule = lgf::kLayoutPlanes;
    // warm-up under the same sustained load, as for the link sweeps
    const auto w0 = std::chrono::steady_clock::now();
    for (int k = 0; k < 2000 && e == hipSuccess; k += 20) {
        for (int j = 0; j < 20; ++j) sweep(dflt);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count() > 3.0) break;
    }
    // FP64 sweep formats keep the blocked tile order wherever the lattice
    // admits it: it reads each neighbouring g about once (counted
    // L2-to-memory traffic 1.06-1.07x the algorithmic bytes at 64^4, against
    // 1.2x for the lockstep order and 1.2-1.4x for the lexicographic one, which
    // are no faster); an order the lattice does not admit would run as order 0
    // and is left out
    const bool fp64 = (format == LGF_FP64_18 || format == LGF_FP64_12 || format == LGF_FP64_12S);
    std::vector<lgf::SweepTuning> variants;
    for (int lps : {1, 2, 4}) {
        if (lps == 1 && !lgf::fixed_one_lane_format(format)) continue;
        for (int block : {64, 128, 256}) {
            lgf::SweepTuning t{};
            t.lanes_per_site = lps;
            t.block = block;
            const bool blocked = fp64 && lgf::fixed_order_admitted(h->geom, t, 2);
            for (int order = 0; order < 4; ++order) {
                if (order >= 2 && !lgf::fixed_order_admitted(h->geom, t, order)) continue;
                if (blocked && order != 2) continue;
                t.xcd_remap = order;
                for (int layout : {lgf::kLayoutPlanes, lgf::kLayoutRecords}) {
                    if (layout == lgf::kLayoutRecords && !records) continue;
                    t.schedule = layout;
                    variants.push_back(t);
                }
            }
        }
    }
    lgf::SweepTuning best = h->tune_fixed[format];
    const bool ok = e == hipSuccess &&
                    pick_variant(variants, dflt, trials, "lgf_autotune_fixed", format, time_variant, &best);
    (void)hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(LGF_EHIP, "autotune_fixed: %s", hipGetErrorString(e));
    if (ok) h->tune_fixed[format] = best;
    drop_graphs(h);
    if (h->rec[format] && !fixed_records(h, format)) {
        // the picked variant reads the link field: the records' memory goes back
        (void)hipFree(h->rec[format]);
        h->rec[format] = nullptr;
    }
    return LGF_OK;
}

lgf_status lgf_autotune(lgf_lattice *h, int format, int trials)
{
    if (!h) return fail(LGF_EINVAL, "handle is NULL");
    h->fix_on = false;
    if (!valid_format(format)) return fail(LGF_EINVAL, "unknown format %d", format);
    if (trials < 1) return fail(LGF_EINVAL, "trials must be >= 1");
    LGF_TRY(use_device(h));
    // The variants sweep the very buffer the gauge fixing sweeps in this
    // format (the handle's field, or its working copy in another format):
    // measured on one GPU the in-place and out-of-place rates depend on the
    // buffer, by a few per cent either way.  The handle's own links are saved
    // before and restored after; a working copy holds no state between calls.
    const size_t bytes = (size_t)h->V * 4 * lgf::link_bytes(format);
    void *scratch = nullptr, *backup = nullptr;
    hipError_t e = hipSuccess;
    if (format == h->format) {
        scratch = h->field;
        if (hipMalloc(&backup, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LGF_ENOMEM, "cannot allocate %zu bytes to save the links while tuning", bytes);
        }
        e = hipMemcpyAsync(backup, h->field, bytes, hipMemcpyDeviceToDevice, h->stream);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(h->stream);
            (void)hipFree(backup);
            return fail(LGF_EHIP, "autotune: saving the links: %s", hipGetErrorString(e));
        }
    } else {
        LGF_TRY(ensure_work(h, format));
        scratch = h->work[format];
        e = lgf::launch_convert(h->format, h->field, format, scratch, h->geom, false, h->stream);
    }
    // the out-of-place variants need the partner buffer; without memory for it
    // they are skipped (and an out-of-place tuning falls back to in place)
    const bool had_partner = h->partner[format] != nullptr;
    const bool can_oop = ensure_partner(h, format) == LGF_OK;
    if (!can_oop && h->tune[format].schedule == lgf::kScheduleOutOfPlace)
        h->tune[format].schedule = lgf::kScheduleInPlace;
    const lgf::SweepTuning saved = h->tune[format];
    lgf_status st = LGF_OK;
    // time n full sweeps of one variant after one untimed full sweep
    auto time_variant = [&](const lgf::SweepTuning &t, int n, double *ms) {
        h->tune[format] = t;
        st = full_sweep(h, format, scratch, 1.7, 0.0, 0, 0);
        if (st != LGF_OK) return false;
        e = hipEventRecord(h->ev0, h->stream);
        for (int k = 0; k < n && e == hipSuccess && st == LGF_OK; ++k)
            st = full_sweep(h, format, scratch, 1.7, 0.0, 0, 0);
        if (e == hipSuccess) e = hipEventRecord(h->ev1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(h->ev1);
        if (e != hipSuccess || st != LGF_OK) return false;
        *ms = elapsed_ms(h->ev0, h->ev1) / n;
        return true;
    };
    // warm-up: the GPU's clocks settle under a sustained streaming load within
    // seconds, and the variants rank differently on a cold GPU (the ones with
    // more arithmetic per byte look better) than in a long gauge fixing
    if (e == hipSuccess) {
        const auto w0 = std::chrono::steady_clock::now();
        for (int k = 0; k < 2000 && st == LGF_OK && e == hipSuccess; k += 20) {
            for (int j = 0; j < 20 && st == LGF_OK; ++j) st = full_sweep(h, format, scratch, 1.7, 0.0, 0, 0);
            e = hipStreamSynchronize(h->stream);
            if (std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count() > 3.0) break;
        }
    }
    // stage 1: every variant once
    std::vector<lgf::SweepTuning> variants;
    const int lps_list[3] = {1, 2, 4};
    const int block_list[3] = {64, 128, 256};
    for (int li = 0; li < 3; ++li)
        for (int bi = 0; bi < 3; ++bi)
            for (int v = 0; v < 48; ++v) {
                const int xcd = v & 1, nt = (v >> 1) & 1, sched = (v >> 2) % 3, spt = 1 << (v / 12);
                // the t-slice pipeline is measured slower at every size it was
                // tried on; it stays a manual option (lgf_set_tuning)
                if (sched == lgf::kSchedulePipeline || spt > 4) continue;
                if (sched == lgf::kScheduleOutOfPlace && (!nt || !can_oop)) continue;
                if (spt > 1 && xcd) continue;
                variants.push_back(lgf::SweepTuning{lps_list[li], block_list[bi], xcd, nt, sched, spt});
            }
    lgf::SweepTuning best = saved;
    if (e == hipSuccess && st == LGF_OK)
        (void)pick_variant(variants, default_tuning(format), trials, "lgf_autotune", format, time_variant, &best);
    h->tune[format] = saved;
    if (backup) {
        const hipError_t e2 = hipMemcpyAsync(h->field, backup, bytes, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = e2;
    }
    (void)hipStreamSynchronize(h->stream);
    if (backup) (void)hipFree(backup);
    if (st == LGF_OK && e == hipSuccess) h->tune[format] = best;
    if (!had_partner && h->partner[format] && h->tune[format].schedule != lgf::kScheduleOutOfPlace) {
        (void)hipFree(h->partner[format]);
        h->partner[format] = nullptr;
    }
    if (st != LGF_OK) return st;
    if (e != hipSuccess) return fail(LGF_EHIP, "autotune: %s", hipGetErrorString(e));
    drop_graphs(h);
    return LGF_OK;
}

lgf_status lgf_time_sweeps(lgf_lattice *h, int n, double omega, double p_sr, uint64_t seed,
                           uint64_t sweep_index, double *ms_per_launch)
{
    if (!h || !ms_per_launch) return fail(LGF_EINVAL, "NULL handle or output");
    h->fix_on = false;
    if (n < 1) return fail(LGF_EINVAL, "n must be >= 1");
    if (!(omega >= 1.0 && omega <= 2.0)) return fail(LGF_EINVAL, "omega %g outside [1, 2]", omega);
    if (!(p_sr >= 0.0 && p_sr <= 1.0)) return fail(LGF_EINVAL, "p_sr %g outside [0, 1]", p_sr);
    LGF_TRY(use_device(h));
    prepare_schedule(h, h->format);
    LGF_HIP(hipEventRecord(h->ev0, h->stream));
    for (int k = 0; k < n; ++k)
        LGF_TRY(full_sweep(h, h->format, h->field, omega, p_sr, seed, sweep_index + (uint64_t)k));
    LGF_HIP(hipEventRecord(h->ev1, h->stream));
    LGF_HIP(hipEventSynchronize(h->ev1));
    *ms_per_launch = elapsed_ms(h->ev0, h->ev1) / (2.0 * n);
    return LGF_OK;
}

}  // extern "C"
