// lgf_fixed.hip -- kernels of the fixed-link form of the relaxation sweep:
// the links keep their input values, the sweep updates the gauge
// transformation g (a site field in the links' format) and forms each link in
// the current gauge, g(x) U_mu(x) g(x+mu)^dag (Eq. (3)), in registers only.
//
// Per site update the stream is 8 links in (read only) plus g(x) in and out,
// and the 8 neighbouring g of the other parity, each shared by 8 sites of the
// half-sweep and mostly served by L2 and the last-level cache: 1056 B of
// unique traffic per site update in FP64-12 against 1536 B for the update that
// rewrites the links, 528 B against 768 B in FP32-12.  The price is the 8
// products U g^dag, g U per site, ~1.3k more multiply-adds, still well under
// the time the bytes take at either precision.
#include "lgf_device.hpp"
#include "lgf_internal.hpp"
#include "lgf_site.hpp"

namespace lgf {

// Order in which the workgroups walk the tiles of a half-sweep (a tile is the
// block / LPS consecutive sites of one workgroup).  Every g of the other
// parity is read by the 8 neighbours of its site, so the order decides how
// often it comes from L2 rather than from HBM: in the lexicographic order the
// y-neighbour rows lie in the next workgroup, which the round-robin dispatch
// puts on another XCD, and the t-neighbours a whole t-slice of tiles away.
//   mode 0: lexicographic;
//   mode 1: contiguous ranges of tiles per XCD;
//   mode 2: blocks of Bt t-slices x Bz z-planes (all y and x) per XCD, each
//           walked with z fastest, then t, then the tiles of a plane, so that
//           the t-, z- and y-neighbours of a tile are 1, Bz and Bt Bz tiles
//           earlier or later on the same XCD.  Block k goes to XCD k % 8 (the
//           dispatch deals workgroup b to XCD b % 8).
//   mode 3: the (t, z) planes in lexicographic order on all XCDs at once, each
//           XCD taking its own eighth of every plane (P / 8 consecutive tiles,
//           P tiles per plane): the y-neighbours of a tile are mostly on its
//           XCD, its z- and t-neighbours were read by the same XCD one plane
//           and one t-slice earlier, and the 8 XCDs stream through the same
//           region of memory together.
struct TileOrder {
    uint32_t mode;
    uint32_t tile;   // sites per tile
    uint32_t P;      // tiles per (t, z) plane
    uint32_t plane;  // sites per (t, z) plane, Ly Lx / 2
    uint32_t Bt, Bz, nzb;  // block extents in t and z; Lz / Bz
    uint32_t tpb;    // tiles per block, Bt Bz P
};

// One half-sweep over all Vh sites of a parity, LPS lanes per site; POST as
// in update_site_fixed, with workgroup b's (F, theta) sums in partials[2b]
// when POST == 2.  MU0 = 1: Coulomb gauge, with the timeslice flags
// slice_active.  REC: the links are per-site link records.
template <int F, int LPS, bool SR, int POST, int MU0 = 0, bool REC = false>
__global__ void __launch_bounds__(256) fixed_sweep_kernel(const void *__restrict__ links, void *__restrict__ gf,
                                                          Geom g, int parity, RelaxArgs<typename Fmt<F>::T> a,
                                                          TileOrder o, uint32_t n_groups,
                                                          double *__restrict__ partials,
                                                          const uint8_t *__restrict__ slice_active)
{
    const uint32_t b = blockIdx.x;
    uint32_t h0;        // first site of the tile (Vh <= 2^30, LPS <= 4)
    uint32_t slot = b;  // partial-sum slot: the tile's index, < n_groups, so
                        // that the final sum does not depend on the order
    if (o.mode == 2) {
        const uint32_t s = b >> 3, blk = (s / o.tpb) * 8u + (b & 7u), i = s % o.tpb;
        const uint32_t r = i % (o.Bt * o.Bz);
        const uint32_t t = (blk / o.nzb) * o.Bt + r / o.Bz, z = (blk % o.nzb) * o.Bz + r % o.Bz;
        h0 = (t * g.L[1] + z) * o.plane + (i / (o.Bt * o.Bz)) * o.tile;
        slot = h0 / o.tile;
    } else if (o.mode == 3) {
        const uint32_t s = b >> 3, G = o.P >> 3;
        h0 = (s / G) * o.plane + ((b & 7u) * G + s % G) * o.tile;
        slot = h0 / o.tile;
    } else if (o.mode == 1) {
        const uint32_t per = gridDim.x >> 3, w = (b & 7u) * per + (b >> 3);
        if (w >= n_groups) return;  // the whole workgroup: no tile
        h0 = w * o.tile;
        slot = w;
    } else {
        h0 = b * o.tile;
    }
    const uint32_t grp = h0 + threadIdx.x / LPS;
    const bool active = grp < g.Vh;
    MeasAcc acc;
    update_site_fixed<F, LPS, SR, POST, MU0, REC>(links, gf, g, parity, active ? grp : g.Vh - 1,
                                             (int)(threadIdx.x % LPS), active, a, &acc, slice_active);
    if constexpr (POST == 2) block_sum2_any(acc.f, acc.th, partials + 2 * slot);
}

uint32_t fixed_sweep_groups(const Geom &g, const SweepTuning &t)
{
    const uint64_t threads = (uint64_t)g.Vh * (uint64_t)t.lanes_per_site;
    return (uint32_t)((threads + t.block - 1) / t.block);
}

// The tile order of a tuning on this lattice; mode 2 takes the largest
// blocks of 8, 4 or 2 t-slices and z-planes that divide the lattice into a
// multiple of 8 blocks of whole tiles, mode 3 needs planes of a multiple of
// 8 whole tiles; otherwise both fall back to mode 0.
static TileOrder tile_order(const Geom &g, const SweepTuning &t)
{
    TileOrder o{};
    o.mode = (uint32_t)t.xcd_remap;
    o.tile = (uint32_t)(t.block / t.lanes_per_site);
    o.plane = g.L[2] * g.hx;
    if (o.mode == 3) {
        o.mode = 0;
        if (o.plane % o.tile != 0 || (o.plane / o.tile) % 8 != 0) return o;
        o.P = o.plane / o.tile;
        o.mode = 3;
        return o;
    }
    if (o.mode != 2) return o;
    o.mode = 0;
    if (o.plane % o.tile != 0) return o;
    o.P = o.plane / o.tile;
    for (uint32_t B = 8; B >= 2; B >>= 1) {
        if (g.L[0] % B != 0 || g.L[1] % B != 0) continue;
        const uint32_t nb = (g.L[0] / B) * (g.L[1] / B);
        if (nb % 8 != 0) continue;
        o.mode = 2;
        o.Bt = o.Bz = B;
        o.nzb = g.L[1] / B;
        o.tpb = B * B * o.P;
        break;
    }
    return o;
}

bool fixed_order_admitted(const Geom &g, const SweepTuning &t, int order)
{
    SweepTuning b = t;
    b.xcd_remap = order;
    return (int)tile_order(g, b).mode == order;
}

template <int F, int LPS, bool REC>
static hipError_t launch_fixed_t(const void *links, void *gf, const Geom &g, const SweepArgs &a, const SweepTuning &t,
                                 int post, const uint8_t *slices, bool coulomb, hipStream_t s)
{
    using T = typename Fmt<F>::T;
    const uint32_t ng = fixed_sweep_groups(g, t);
    const TileOrder o = tile_order(g, t);
    const dim3 grid(o.mode == 1 ? ((ng + 7u) / 8u) * 8u : ng), block(t.block);
    RelaxArgs<T> ra{(T)a.omega, (a.omega != 1.0) ? 1 : 0, 0, (uint32_t)a.seed, (uint32_t)(a.seed >> 32),
                    (uint32_t)a.sweep_index, a.instance, nullptr, a.sweep_base};
    const bool sr = a.p_sr > 0.0;
    if (sr) ra.sr_threshold = (uint64_t)floor(a.p_sr * 4294967296.0);
    double *m = a.meas;
    if (post == 2 && (!m || coulomb)) return hipErrorInvalidValue;
#define LGF_FIX_LAUNCH(SRV, P) \
    hipLaunchKernelGGL((fixed_sweep_kernel<F, LPS, SRV, P, 0, REC>), grid, block, 0, s, links, gf, g, a.parity, ra, o, \
                       ng, m, nullptr)
#define LGF_FIX_LAUNCH_C(SRV, P) \
    hipLaunchKernelGGL((fixed_sweep_kernel<F, LPS, SRV, P, 1, REC>), grid, block, 0, s, links, gf, g, a.parity, ra, o, \
                       ng, nullptr, slices)
    if (coulomb) {
        if (sr) {
            if (post == 0) LGF_FIX_LAUNCH_C(true, 0);
            else LGF_FIX_LAUNCH_C(true, 1);
        } else {
            if (post == 0) LGF_FIX_LAUNCH_C(false, 0);
            else LGF_FIX_LAUNCH_C(false, 1);
        }
    } else if (sr) {
        if (post == 0) LGF_FIX_LAUNCH(true, 0);
        else if (post == 1) LGF_FIX_LAUNCH(true, 1);
        else LGF_FIX_LAUNCH(true, 2);
    } else {
        if (post == 0) LGF_FIX_LAUNCH(false, 0);
        else if (post == 1) LGF_FIX_LAUNCH(false, 1);
        else LGF_FIX_LAUNCH(false, 2);
    }
#undef LGF_FIX_LAUNCH
#undef LGF_FIX_LAUNCH_C
    return hipGetLastError();
}

// per-site link records: the 12-real formats and the split storage
bool fixed_records_format(int format) { return format == kF32_12 || format == kF64_12 || format == kF64_12S; }
// one lane per site: the FP32 formats (in FP64 the update takes all 512
// registers and runs one wave per SIMD, slower than two lanes per site)
bool fixed_one_lane_format(int format) { return format == kF32_12 || format == kF32_18; }

template <int F, bool REC>
static hipError_t launch_fixed_r(const void *links, void *gf, const Geom &g, const SweepArgs &a, const SweepTuning &t,
                                 int post, const uint8_t *slices, bool coulomb, hipStream_t s)
{
    switch (t.lanes_per_site) {
    case 1:
        if constexpr (F == kF32_12 || F == kF32_18)
            return launch_fixed_t<F, 1, REC>(links, gf, g, a, t, post, slices, coulomb, s);
        else
            return hipErrorInvalidValue;
    case 2: return launch_fixed_t<F, 2, REC>(links, gf, g, a, t, post, slices, coulomb, s);
    case 4: return launch_fixed_t<F, 4, REC>(links, gf, g, a, t, post, slices, coulomb, s);
    default: return hipErrorInvalidValue;
    }
}

template <int F>
static hipError_t launch_fixed_f(const void *links, void *gf, const Geom &g, const SweepArgs &a, const SweepTuning &t,
                                 int post, const uint8_t *slices, bool coulomb, hipStream_t s)
{
    if (t.schedule == kLayoutRecords) {
        if constexpr (F == kF32_12 || F == kF64_12 || F == kF64_12S)
            return launch_fixed_r<F, true>(links, gf, g, a, t, post, slices, coulomb, s);
        else
            return hipErrorInvalidValue;
    }
    return launch_fixed_r<F, false>(links, gf, g, a, t, post, slices, coulomb, s);
}

static hipError_t launch_fixed_any(int format, const void *links, void *gf, const Geom &g, const SweepArgs &a,
                                   const SweepTuning &t, int post, const uint8_t *slices, bool coulomb, hipStream_t s)
{
    if (t.block <= 0 || t.block > 256 || (t.block % 64) != 0 || post < 0 || post > 2 || a.h_end != 0 || a.out ||
        (t.schedule != kLayoutPlanes && t.schedule != kLayoutRecords))
        return hipErrorInvalidValue;
    switch (format) {
    case kF64_18: return launch_fixed_f<kF64_18>(links, gf, g, a, t, post, slices, coulomb, s);
    case kF32_18: return launch_fixed_f<kF32_18>(links, gf, g, a, t, post, slices, coulomb, s);
    case kF32_12: return launch_fixed_f<kF32_12>(links, gf, g, a, t, post, slices, coulomb, s);
    case kF64_12: return launch_fixed_f<kF64_12>(links, gf, g, a, t, post, slices, coulomb, s);
    case kF64_12S: return launch_fixed_f<kF64_12S>(links, gf, g, a, t, post, slices, coulomb, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fixed_sweep(int format, const void *links, void *gf, const Geom &g, const SweepArgs &a,
                              const SweepTuning &t, int post, hipStream_t s)
{
    return launch_fixed_any(format, links, gf, g, a, t, post, nullptr, false, s);
}

hipError_t launch_fixed_sweep_coulomb(int format, const void *links, void *gf, const Geom &g, const SweepArgs &a,
                                      const SweepTuning &t, int post, const uint8_t *slice_active, hipStream_t s)
{
    return launch_fixed_any(format, links, gf, g, a, t, post, slice_active, true, s);
}

// Read-only F / theta pass of the fixed-link form: 2 lanes per site,
// kMeasureBlock lanes per workgroup, one (F, theta) partial pair per workgroup.
constexpr int kMeasureFixedLanes = 2;

int fixed_measure_blocks(const Geom &g)
{
    return (int)(((uint64_t)g.Vh * kMeasureFixedLanes + kMeasureBlock - 1) / kMeasureBlock);
}

template <int F, bool REC = false>
__global__ void __launch_bounds__(kMeasureBlock) measure_fixed_kernel(const void *__restrict__ links,
                                                                      const void *__restrict__ gf, Geom g,
                                                                      int parity, double *partials)
{
    const uint32_t tid = blockIdx.x * kMeasureBlock + threadIdx.x;
    const uint32_t h0 = tid / kMeasureFixedLanes;
    const bool active = h0 < g.Vh;
    double f, th;
    measure_site_fixed<F, kMeasureFixedLanes, 0, REC>(links, gf, g, parity, active ? h0 : g.Vh - 1,
                                                      (int)(tid % kMeasureFixedLanes), active, f, th);
    block_sum2<kMeasureBlock>(f, th, partials + 2 * blockIdx.x);
}

hipError_t launch_measure_fixed(int format, const void *links, const void *gf, const Geom &g, int parity,
                                double *partials, int *n_partials, hipStream_t s, bool records)
{
    const int nb = fixed_measure_blocks(g);
    *n_partials = nb;
    const dim3 grid(nb), block(kMeasureBlock);
    if (records) {
        switch (format) {
        case kF32_12: hipLaunchKernelGGL((measure_fixed_kernel<kF32_12, true>), grid, block, 0, s, links, gf, g, parity, partials); break;
        case kF64_12: hipLaunchKernelGGL((measure_fixed_kernel<kF64_12, true>), grid, block, 0, s, links, gf, g, parity, partials); break;
        case kF64_12S: hipLaunchKernelGGL((measure_fixed_kernel<kF64_12S, true>), grid, block, 0, s, links, gf, g, parity, partials); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (format) {
    case kF64_18: hipLaunchKernelGGL((measure_fixed_kernel<kF64_18>), grid, block, 0, s, links, gf, g, parity, partials); break;
    case kF32_18: hipLaunchKernelGGL((measure_fixed_kernel<kF32_18>), grid, block, 0, s, links, gf, g, parity, partials); break;
    case kF32_12: hipLaunchKernelGGL((measure_fixed_kernel<kF32_12>), grid, block, 0, s, links, gf, g, parity, partials); break;
    case kF64_12: hipLaunchKernelGGL((measure_fixed_kernel<kF64_12>), grid, block, 0, s, links, gf, g, parity, partials); break;
    case kF64_12S: hipLaunchKernelGGL((measure_fixed_kernel<kF64_12S>), grid, block, 0, s, links, gf, g, parity, partials); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Coulomb gauge, read only: per timeslice t and parity pass, partial (F_C,
// theta_C) pairs at partials[2 (t bps + b)] for the bps = coulomb_fixed_blocks
// workgroups of a slice (the layout finish_coulomb_kernel sums).
int coulomb_fixed_blocks(const Geom &g)
{
    return (int)(((uint64_t)g.hs[0] * kMeasureFixedLanes + kMeasureBlock - 1) / kMeasureBlock);
}

template <int F, bool REC = false>
__global__ void __launch_bounds__(kMeasureBlock) measure_coulomb_fixed_kernel(const void *__restrict__ links,
                                                                              const void *__restrict__ gf, Geom g,
                                                                              int parity, double *partials)
{
    const uint32_t t = blockIdx.y;
    const uint32_t tid = blockIdx.x * kMeasureBlock + threadIdx.x;
    const uint32_t i = tid / kMeasureFixedLanes;
    const bool active = i < g.hs[0];
    const uint32_t h = t * g.hs[0] + (active ? i : g.hs[0] - 1);
    double f, th;
    measure_site_fixed<F, kMeasureFixedLanes, 1, REC>(links, gf, g, parity, h, (int)(tid % kMeasureFixedLanes),
                                                      active, f, th);
    block_sum2<kMeasureBlock>(f, th, partials + 2 * ((size_t)t * gridDim.x + blockIdx.x));
}

hipError_t launch_measure_coulomb_fixed(int format, const void *links, const void *gf, const Geom &g, int parity,
                                        double *partials, hipStream_t s, bool records)
{
    const dim3 grid(coulomb_fixed_blocks(g), g.L[0]), block(kMeasureBlock);
    if (records) {
        switch (format) {
        case kF32_12: hipLaunchKernelGGL((measure_coulomb_fixed_kernel<kF32_12, true>), grid, block, 0, s, links, gf, g, parity, partials); break;
        case kF64_12: hipLaunchKernelGGL((measure_coulomb_fixed_kernel<kF64_12, true>), grid, block, 0, s, links, gf, g, parity, partials); break;
        case kF64_12S: hipLaunchKernelGGL((measure_coulomb_fixed_kernel<kF64_12S, true>), grid, block, 0, s, links, gf, g, parity, partials); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (format) {
    case kF64_18: hipLaunchKernelGGL((measure_coulomb_fixed_kernel<kF64_18>), grid, block, 0, s, links, gf, g, parity, partials); break;
    case kF32_18: hipLaunchKernelGGL((measure_coulomb_fixed_kernel<kF32_18>), grid, block, 0, s, links, gf, g, parity, partials); break;
    case kF32_12: hipLaunchKernelGGL((measure_coulomb_fixed_kernel<kF32_12>), grid, block, 0, s, links, gf, g, parity, partials); break;
    case kF64_12: hipLaunchKernelGGL((measure_coulomb_fixed_kernel<kF64_12>), grid, block, 0, s, links, gf, g, parity, partials); break;
    case kF64_12S: hipLaunchKernelGGL((measure_coulomb_fixed_kernel<kF64_12S>), grid, block, 0, s, links, gf, g, parity, partials); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// site field conversion with FP64 reunitarization (the gauge transformation
// handed from the bulk precision to the finish precision)
template <int FS, int FD>
__global__ void __launch_bounds__(256) site_convert_kernel(const void *__restrict__ src, void *__restrict__ dst,
                                                           uint32_t Vh)
{
    const uint32_t h = blockIdx.x * 256 + threadIdx.x;
    if (h >= Vh) return;
    const int parity = blockIdx.y;
    mat3<typename Fmt<FS>::T> a;
    load_link<FS>(a, site_field_ptr<FS>(const_cast<void *>(src), Vh, parity), Vh, h);
    mat3<double> d;
    convert(d, a);
    reunitarize(d);
    mat3<typename Fmt<FD>::T> o;
    convert(o, d);
    store_link<FD>(site_field_ptr<FD>(dst, Vh, parity), Vh, h, o);
}

template <int FS>
static hipError_t launch_site_convert_s(const void *src, int fd, void *dst, uint32_t Vh, hipStream_t s)
{
    const dim3 grid((Vh + 255) / 256, 2);
    switch (fd) {
    case kF64_18: hipLaunchKernelGGL((site_convert_kernel<FS, kF64_18>), grid, dim3(256), 0, s, src, dst, Vh); break;
    case kF32_18: hipLaunchKernelGGL((site_convert_kernel<FS, kF32_18>), grid, dim3(256), 0, s, src, dst, Vh); break;
    case kF32_12: hipLaunchKernelGGL((site_convert_kernel<FS, kF32_12>), grid, dim3(256), 0, s, src, dst, Vh); break;
    case kF64_12: hipLaunchKernelGGL((site_convert_kernel<FS, kF64_12>), grid, dim3(256), 0, s, src, dst, Vh); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_site_convert(int fs, const void *src, int fd, void *dst, const Geom &g, hipStream_t s)
{
    if (src == dst) return hipErrorInvalidValue;
    switch (fs) {
    case kF64_18: return launch_site_convert_s<kF64_18>(src, fd, dst, g.Vh, s);
    case kF32_18: return launch_site_convert_s<kF32_18>(src, fd, dst, g.Vh, s);
    case kF32_12: return launch_site_convert_s<kF32_12>(src, fd, dst, g.Vh, s);
    case kF64_12: return launch_site_convert_s<kF64_12>(src, fd, dst, g.Vh, s);
    default: return hipErrorInvalidValue;
    }
}

// A link field of the 12-real format F (planes) into per-site link records:
// one lane per (site, parity); the stores of a wavefront are contiguous.
template <int F>
__global__ void __launch_bounds__(256) record_links_kernel(const void *__restrict__ src, void *__restrict__ rec,
                                                           Geom g)
{
    using V = typename Fmt<F>::V;
    constexpr int NV = Fmt<F>::NV;
    const uint32_t h = blockIdx.x * 256 + threadIdx.x;
    if (h >= g.Vh) return;
    const int parity = blockIdx.y;
    const Site c = decode(g, parity, h);
    void *L = const_cast<void *>(src);
    V *out = const_cast<V *>(rec_ptr<F>(rec, g.Vh, parity, 0, h));
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const V *f = block_ptr<F>(L, g.Vh, parity, mu) + h;
        const V *b = block_ptr<F>(L, g.Vh, parity ^ 1, mu) + back_half(g, c, h, mu);
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            out[((size_t)mu * NV + k) * kRecTile] = f[(size_t)k * g.Vh];
            out[((size_t)(4 + mu) * NV + k) * kRecTile] = b[(size_t)k * g.Vh];
        }
    }
}

// the same for the split storage of kF64_12S (src as launch_split_links
// writes it): both parts of every link copied as they are
__global__ void __launch_bounds__(256) record_split_links_kernel(const void *__restrict__ src, void *__restrict__ rec,
                                                                 Geom g)
{
    const uint32_t h = blockIdx.x * 256 + threadIdx.x;
    if (h >= g.Vh) return;
    const int parity = blockIdx.y;
    const Site c = decode(g, parity, h);
    void *L = const_cast<void *>(src);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const uint32_t hb = back_half(g, c, h, mu);
        const v4f *fh = block_ptr<kF32_12>(L, g.Vh, parity, mu) + h;
        const v4s *fq = split_res_ptr(L, g.Vh, parity, mu) + h;
        const v4f *bh = block_ptr<kF32_12>(L, g.Vh, parity ^ 1, mu) + hb;
        const v4s *bq = split_res_ptr(L, g.Vh, parity ^ 1, mu) + hb;
        v4f *ofh = const_cast<v4f *>(rec_split_hi(rec, g.Vh, parity, mu, h));
        v4s *ofq = const_cast<v4s *>(rec_split_lo(rec, g.Vh, parity, mu, h));
        v4f *obh = const_cast<v4f *>(rec_split_hi(rec, g.Vh, parity, 4 + mu, h));
        v4s *obq = const_cast<v4s *>(rec_split_lo(rec, g.Vh, parity, 4 + mu, h));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ofh[(size_t)k * kRecTile] = fh[(size_t)k * g.Vh];
            ofq[(size_t)k * kRecTile] = fq[(size_t)k * g.Vh];
            obh[(size_t)k * kRecTile] = bh[(size_t)k * g.Vh];
            obq[(size_t)k * kRecTile] = bq[(size_t)k * g.Vh];
        }
    }
}

size_t record_links_bytes(int format, const Geom &g)
{
    if (!fixed_records_format(format)) return 0;
    const size_t link = (format == kF64_12) ? 96 : (format == kF64_12S) ? 72 : 48;
    return (size_t)2 * rec_tiles(g.Vh) * kRecTile * 8 * link;
}

hipError_t launch_record_links(int format, const void *src, void *rec, const Geom &g, hipStream_t s)
{
    const dim3 grid((g.Vh + 255) / 256, 2), block(256);
    switch (format) {
    case kF32_12: hipLaunchKernelGGL((record_links_kernel<kF32_12>), grid, block, 0, s, src, rec, g); break;
    case kF64_12: hipLaunchKernelGGL((record_links_kernel<kF64_12>), grid, block, 0, s, src, rec, g); break;
    case kF64_12S: hipLaunchKernelGGL(record_split_links_kernel, grid, block, 0, s, src, rec, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// FP64 links (format fs, a link field) into the split storage of kF64_12S:
// one lane per link of block (parity, mu) = blockIdx.y
template <int FS>
__global__ void __launch_bounds__(256) split_links_kernel(const void *__restrict__ src, void *__restrict__ dst,
                                                          uint32_t Vh)
{
    const uint32_t h = blockIdx.x * 256 + threadIdx.x;
    if (h >= Vh) return;
    const int parity = (int)(blockIdx.y >> 2), mu = (int)(blockIdx.y & 3);
    mat3<double> u;
    load_link<FS, true, false>(u, block_ptr<FS>(const_cast<void *>(src), Vh, parity, mu), Vh, h);
    v4f *hb = block_ptr<kF32_12>(dst, Vh, parity, mu);
    v4s *qb = split_res_ptr(dst, Vh, parity, mu);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const cpx<double> a = u.e[(2 * k) / 3][(2 * k) % 3], b = u.e[(2 * k + 1) / 3][(2 * k + 1) % 3];
        v4f hi;
        v4s q;
        float f;
        short r;
        split_encode(a.re, f, r); hi.x = f; q.x = r;
        split_encode(a.im, f, r); hi.y = f; q.y = r;
        split_encode(b.re, f, r); hi.z = f; q.z = r;
        split_encode(b.im, f, r); hi.w = f; q.w = r;
        vstore<true>(hb + (size_t)k * Vh + h, hi);
        vstore<true>(qb + (size_t)k * Vh + h, q);
    }
}

size_t split_links_bytes(const Geom &g) { return (size_t)g.Vh * 24 * (16 + 8); }

hipError_t launch_split_links(int fs, const void *src, void *dst, const Geom &g, hipStream_t s)
{
    const dim3 grid((g.Vh + 255) / 256, 8);
    switch (fs) {
    case kF64_18: hipLaunchKernelGGL((split_links_kernel<kF64_18>), grid, dim3(256), 0, s, src, dst, g.Vh); break;
    case kF64_12: hipLaunchKernelGGL((split_links_kernel<kF64_12>), grid, dim3(256), 0, s, src, dst, g.Vh); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lgf
