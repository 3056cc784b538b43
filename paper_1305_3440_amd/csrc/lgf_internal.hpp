// lgf_internal.hpp -- host-side launchers of the gfx950 kernels (defined in
// lgf_kernels.hip) as seen by the C-ABI runtime (lgf_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace lgf {

struct Geom;

// bytes of one link in a storage format, and vector slots per link
size_t link_bytes(int format);

struct SweepTuning {
    int lanes_per_site = 1;  // 1, 2 or 4
    int block = 128;         // threads per workgroup (fastest measured at 64^4)
    int xcd_remap = 0;       // contiguous workgroup ranges per XCD
    int nontemporal = 1;     // stream links past the caches
    int schedule = 0;        // full sweeps: 0 two in-place launches, 1 t-slice pipeline
                             // (parity 1 one slice behind), 2 out of place (ping-pong
                             // between the field and a second buffer of its format)
    int sites_per_thread = 1;  // tiles per workgroup (1, 2 or 4), strided over the launch
};

constexpr int kScheduleInPlace = 0, kSchedulePipeline = 1, kScheduleOutOfPlace = 2;
// the fixed-link sweep's `schedule`: layout of the links it reads
constexpr int kLayoutPlanes = 0, kLayoutRecords = 1;

inline bool operator==(const SweepTuning &a, const SweepTuning &b)
{
    return a.lanes_per_site == b.lanes_per_site && a.block == b.block && a.xcd_remap == b.xcd_remap &&
           a.nontemporal == b.nontemporal && a.schedule == b.schedule && a.sites_per_thread == b.sites_per_thread;
}

struct SweepArgs {
    int parity;
    double omega;
    double p_sr;
    uint64_t seed;
    uint64_t sweep_index;
    uint32_t instance;
    uint32_t h_begin = 0;    // half-index range of the launch; h_end = 0: all Vh
    uint32_t h_end = 0;
    void *gacc = nullptr;    // site field accumulating G (same format as the links), or none
    void *out = nullptr;     // out-of-place target field (whole half-sweep only), or in place
    double *meas = nullptr;  // fused reunitarize + measure: per-workgroup (F, theta) partial sums
    const uint64_t *sweep_base = nullptr;  // SR counter = *sweep_base + sweep_index when set
};

// *p = v, as a one-lane kernel on the stream (safe inside a captured graph)
hipError_t launch_set_u64(uint64_t *p, uint64_t v, hipStream_t s);

// workgroups of a whole half-sweep with tuning t (the partial sums a fused
// measurement writes)
uint32_t sweep_groups(const Geom &g, const SweepTuning &t);

hipError_t launch_sweep(int format, void *field, const Geom &g, const SweepArgs &a,
                        const SweepTuning &t, hipStream_t s);

// Reunitarize (optional) + per-block partial sums of (sum Re tr U, sum |Delta|^2)
// over the sites of one parity.  reunit_fwd: reunitarize the 4 forward links
// of every site and store them; reunit_bwd: reunitarize the backward links in
// registers only (for the first parity pass, whose backward links are the
// other parity's not yet reunitarized forward links).
// Returns the number of partial pairs written in *n_partials.
hipError_t launch_measure(int format, void *field, const Geom &g, int parity, bool reunit_fwd,
                          bool reunit_bwd, double *partials, int *n_partials, hipStream_t s);
int measure_blocks(const Geom &g);

// out[0] = F, out[1] = theta from n partial pairs
hipError_t launch_finish_measure(const double *partials, int n, double V, double *out,
                                 hipStream_t s);

// dst (format fd) <- src (format fs), optionally reunitarized in FP64; src may
// equal dst when the formats are equal (element-wise in place).
hipError_t launch_convert(int fs, const void *src, int fd, void *dst, const Geom &g, bool reunit,
                          hipStream_t s);

hipError_t launch_generate(int format, void *field, const Geom &g, uint64_t seed, double eps,
                           bool haar, hipStream_t s);

// canonical double[n][4][18] chunk for sites [s0, s0+n) <-> field
hipError_t launch_canon_to_field(int format, const double *canon, int64_t s0, int64_t n,
                                 void *field, const Geom &g, hipStream_t s);
hipError_t launch_field_to_canon(int format, const void *field, const int64_t *sites, int64_t s0,
                                 int64_t n, double *canon, const Geom &g, hipStream_t s);

// Coulomb gauge (K from the spatial links, per-timeslice masks and sums).
// slice_active: device array of Lt flags (NULL = every timeslice).
hipError_t launch_sweep_coulomb(int format, void *field, const Geom &g, const SweepArgs &a,
                                const uint8_t *slice_active, bool nt, hipStream_t s);
// partials must hold 4 * Lt * coulomb_blocks_per_slice(g) doubles; pass 0
// writes the first half (parity 0 at partials, parity 1 at the second half is
// the caller's offset 2 * Lt * blocks)
int coulomb_blocks_per_slice(const Geom &g);
hipError_t launch_measure_coulomb(int format, void *field, const Geom &g, int parity, bool reunit_fwd,
                                  bool reunit_bwd, double *partials, hipStream_t s);
// bps: partial pairs per timeslice and pass (coulomb_blocks_per_slice or
// coulomb_fixed_blocks)
hipError_t launch_finish_coulomb(const double *partials, const Geom &g, int bps, double *out, hipStream_t s);

// site field (2 parities x one SU(3) per site, link-direction layout):
// mode 0 sets the identity, mode 1 reunitarizes in FP64
hipError_t launch_site_field(int format, void *gf, const Geom &g, int mode, hipStream_t s);
// dst (format fd, FP64) <- g(x) src_mu(x) g(x+mu)^dag for src FP64 and g in
// any format (reunitarized in FP64 as it is read); dst may be src
hipError_t launch_gauge_transform(int fs, const void *src, int fg, const void *gf, int fd, void *dst,
                                  const Geom &g, hipStream_t s);

// per-block partial sums of Re tr over the 6 plaquettes of every site (first
// entry of each pair); finish with launch_finish_measure (out[0] * 12 V / 18 V)
hipError_t launch_plaquette(int format, void *field, const Geom &g, double *partials, int *n_partials,
                            hipStream_t s);

// Fixed-link form of the sweep (links read only, the site field gf of the
// gauge transformation updated; both in `format`, or for kF64_12S gf in
// FP64-12 and the links in the split storage of launch_split_links).  post: 0
// plain, 1 the new g reunitarized in FP64 as it is stored, 2 as 1 plus the
// per-workgroup (F, theta) partial sums of the updated sites in a.meas.
// Tuning: lanes per site (1 in the FP32 formats, 2, 4), block, xcd_remap =
// tile order (0..3), schedule = link layout (kLayoutRecords: links holds the
// per-site records of launch_record_links, 12-real formats).
hipError_t launch_fixed_sweep(int format, const void *links, void *gf, const Geom &g, const SweepArgs &a,
                              const SweepTuning &t, int post, hipStream_t s);
uint32_t fixed_sweep_groups(const Geom &g, const SweepTuning &t);
// whether tile order `order` (2: blocks of t-slices x z-planes per XCD; 3:
// an eighth of every plane per XCD) applies to this lattice with the
// tuning's tile size (else the launch falls back to order 0)
bool fixed_order_admitted(const Geom &g, const SweepTuning &t, int order);
// formats with per-site link records; formats that run one lane per site
bool fixed_records_format(int format);
bool fixed_one_lane_format(int format);
// the per-site link records of a 12-real link field src (format, planes):
// record_links_bytes(format, g) bytes at rec (0 for other formats)
size_t record_links_bytes(int format, const Geom &g);
hipError_t launch_record_links(int format, const void *src, void *rec, const Geom &g, hipStream_t s);
// Coulomb gauge in the fixed-link form (post 0 or 1; slice_active: device
// array of Lt flags)
hipError_t launch_fixed_sweep_coulomb(int format, const void *links, void *gf, const Geom &g, const SweepArgs &a,
                                      const SweepTuning &t, int post, const uint8_t *slice_active, hipStream_t s);
// per-timeslice partial (F_C, theta_C) pairs of one parity pass, fixed-link
// form: Lt x coulomb_fixed_blocks(g) pairs, summed by launch_finish_coulomb
int coulomb_fixed_blocks(const Geom &g);
hipError_t launch_measure_coulomb_fixed(int format, const void *links, const void *gf, const Geom &g, int parity,
                                        double *partials, hipStream_t s, bool records);
// per-block (F, theta) partial sums over one parity's sites, fixed-link form;
// *n_partials = fixed_measure_blocks(g) pairs; records: links holds per-site
// link records
int fixed_measure_blocks(const Geom &g);
hipError_t launch_measure_fixed(int format, const void *links, const void *gf, const Geom &g, int parity,
                                double *partials, int *n_partials, hipStream_t s, bool records);
// site field dst (format fd) <- src (format fs), reunitarized in FP64
hipError_t launch_site_convert(int fs, const void *src, int fd, void *dst, const Geom &g, hipStream_t s);
// FP64 link field src (format fs, kF64_18 or kF64_12) into the split storage
// dst of kF64_12S, split_links_bytes(g) bytes
size_t split_links_bytes(const Geom &g);
hipError_t launch_split_links(int fs, const void *src, void *dst, const Geom &g, hipStream_t s);

// Simulated annealing: one heat-bath half-sweep of the link-rewriting form at
// temperature temp > 0 (FP64 formats only).  trials (device counter, may be
// NULL) accumulates the accept-reject trials of the launch.
hipError_t launch_anneal(int format, void *field, const Geom &g, int parity, double temp, uint64_t seed,
                         uint64_t sweep, uint32_t instance, unsigned long long *trials, hipStream_t s);

}  // namespace lgf
