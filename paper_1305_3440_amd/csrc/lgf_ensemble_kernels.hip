// lgf_ensemble_kernels.hip -- persistent kernels that sweep and measure an
// ensemble of independent lattices of different sizes in one launch.
//
// The work list is a flat array of tiles (configuration, first half index):
// every tile is `tile` sites of one configuration (64, 128 or 256, one lane per
// site and one workgroup per tile; at 128 a 24^4 lattice contributes 1296 tiles
// per parity and an 8^4 one 16).  A fixed grid of workgroups (a few per CU)
// walks the list; each tile reads its configuration's descriptor
// (geometry, field pointer, current storage format) and runs the same per-site
// update as the single-lattice sweep.  Converged configurations are simply
// left out of the list, and a configuration in its FP32 bulk phase and one in
// its FP64 finish phase share the launch.  The list length, the descriptors
// and the sweep counter live in device memory, so a captured graph of sweep
// launches stays valid while the work list changes between chunks.
#include "lgf_device.hpp"
#include "lgf_ensemble.hpp"
#include "lgf_site.hpp"

namespace lgf {

template <int F, bool SR, bool NT, bool MEAS>
__device__ __forceinline__ void ensemble_site(const EnsCfg &c, int parity, uint32_t h, bool active,
                                              const EnsRelax &r, uint32_t sweep, MeasAcc *acc)
{
    using T = typename Fmt<F>::T;
    const RelaxArgs<T> a{(T)r.omega, r.overrelax, r.sr_threshold, r.key0, r.key1, sweep, c.instance};
    update_site<F, 1, SR, NT, 0, false, false, MEAS>(c.field, c.g, parity, h, 0, active, a, nullptr, nullptr, acc);
}

// FA, FB: the (at most two) storage formats the launch may meet.  MEAS: the
// links are reunitarized as they are written and each tile t leaves its
// sites' (F, theta) sums in partials[2 (n + t)], the second-pass slots of the
// ensemble measurement's layout (n = the listed tiles).
template <int FA, int FB, bool SR, bool NT, bool MEAS = false>
__global__ void __launch_bounds__(kEnsMaxTile) ensemble_sweep_kernel(const EnsCfg *__restrict__ cfgs,
                                                                   const EnsTile *__restrict__ tiles,
                                                                   const uint32_t *__restrict__ n_tiles,
                                                                   const uint64_t *__restrict__ sweep_base,
                                                                   int parity, EnsRelax r, uint32_t sweep_offset,
                                                                   double *__restrict__ partials)
{
    const uint32_t n = *n_tiles;
    const uint32_t sweep = (uint32_t)(*sweep_base + sweep_offset);
    for (uint32_t t = blockIdx.x; t < n; t += gridDim.x) {
        const EnsTile w = tiles[t];
        const EnsCfg c = cfgs[w.cfg];
        const uint32_t h0 = w.h0 + threadIdx.x;
        const bool active = h0 < c.g.Vh;
        const uint32_t h = active ? h0 : c.g.Vh - 1;
        MeasAcc acc;
        if (c.fmt == FA) ensemble_site<FA, SR, NT, MEAS>(c, parity, h, active, r, sweep, &acc);
        else if (FB != FA && c.fmt == FB) ensemble_site<FB, SR, NT, MEAS>(c, parity, h, active, r, sweep, &acc);
        if constexpr (MEAS) {
            block_sum2_any(acc.f, acc.th, partials + 2 * ((size_t)n + t));
            __syncthreads();  // the block sum's shared slots are reused by the next tile
        }
    }
}

template <int FA, int FB>
__global__ void __launch_bounds__(kEnsMaxTile) ensemble_measure_kernel(const EnsCfg *__restrict__ cfgs,
                                                                     const EnsTile *__restrict__ tiles,
                                                                     int parity, int reunit_fwd, int reunit_bwd,
                                                                     double *partials)
{
    const EnsTile w = tiles[blockIdx.x];
    const EnsCfg c = cfgs[w.cfg];
    const uint32_t h0 = w.h0 + threadIdx.x;
    const bool active = h0 < c.g.Vh;
    const uint32_t h = active ? h0 : c.g.Vh - 1;
    double f = 0.0, th = 0.0;
    if (c.fmt == FA) measure_site<FA>(c.field, c.g, parity, h, active, reunit_fwd, reunit_bwd, f, th);
    else if (FB != FA && c.fmt == FB) measure_site<FB>(c.field, c.g, parity, h, active, reunit_fwd, reunit_bwd, f, th);
    block_sum2_any(f, th, partials + 2 * blockIdx.x);
}

// One workgroup per listed configuration: the sums of its tiles' partials
// from both parity passes, in a fixed order, normalised to F and theta.
__global__ void __launch_bounds__(256) ensemble_finish_kernel(const double *__restrict__ partials,
                                                              uint32_t n_tiles,
                                                              const EnsSpan *__restrict__ spans,
                                                              double *__restrict__ out)
{
    const EnsSpan sp = spans[blockIdx.x];
    double a = 0.0, b = 0.0;
    for (uint32_t pass = 0; pass < 2; ++pass)
        for (uint32_t i = threadIdx.x; i < sp.count; i += 256) {
            const double *p = partials + 2 * ((size_t)pass * n_tiles + sp.first + i);
            a += p[0];
            b += p[1];
        }
    __shared__ double r[2];
    block_sum2<256>(a, b, r);
    if (threadIdx.x == 0) {
        out[2 * sp.cfg] = r[0] / (12.0 * sp.V);
        out[2 * sp.cfg + 1] = r[1] / (3.0 * sp.V);
    }
}

// ----------------------------------------------------------------------------
// Fixed-link form: the links stay as stored, each configuration's gauge
// transformation cfgs[].gf is updated (update_site_fixed, 2 lanes per site).
// ----------------------------------------------------------------------------

// REC: the links come from the configuration's per-site records
template <int F, bool SR, int POST, bool REC>
__device__ __forceinline__ void ensemble_site_fixed(const EnsCfg &c, int parity, uint32_t h, int lane, bool active,
                                                    const EnsRelax &r, uint32_t sweep, MeasAcc *acc)
{
    using T = typename Fmt<F>::T;
    const RelaxArgs<T> a{(T)r.omega, r.overrelax, r.sr_threshold, r.key0, r.key1, sweep, c.instance};
    update_site_fixed<F, kEnsFixedLanes, SR, POST, 0, REC>(REC ? c.rec : c.field, c.gf, c.g, parity, h, lane, active,
                                                          a, acc);
}

template <int FA, int FB, bool SR, int POST, bool REC>
__global__ void __launch_bounds__(kEnsMaxTile) ensemble_fixed_kernel(const EnsCfg *__restrict__ cfgs,
                                                                   const EnsTile *__restrict__ tiles,
                                                                   const uint32_t *__restrict__ n_tiles,
                                                                   const uint64_t *__restrict__ sweep_base,
                                                                   int parity, EnsRelax r, uint32_t sweep_offset,
                                                                   double *__restrict__ partials)
{
    const uint32_t n = *n_tiles;
    const uint32_t sweep = (uint32_t)(*sweep_base + sweep_offset);
    const int lane = (int)(threadIdx.x % kEnsFixedLanes);
    for (uint32_t t = blockIdx.x; t < n; t += gridDim.x) {
        const EnsTile w = tiles[t];
        const EnsCfg c = cfgs[w.cfg];
        const uint32_t h0 = w.h0 + threadIdx.x / kEnsFixedLanes;
        const bool active = h0 < c.g.Vh;
        const uint32_t h = active ? h0 : c.g.Vh - 1;
        MeasAcc acc;
        if (c.fmt == FA) ensemble_site_fixed<FA, SR, POST, REC>(c, parity, h, lane, active, r, sweep, &acc);
        else if (FB != FA && c.fmt == FB)
            ensemble_site_fixed<FB, SR, POST, REC>(c, parity, h, lane, active, r, sweep, &acc);
        if constexpr (POST == 2) {
            block_sum2_any(acc.f, acc.th, partials + 2 * ((size_t)n + t));
            __syncthreads();  // the block sum's shared slots are reused by the next tile
        }
    }
}

template <int FA, int FB, bool REC>
__global__ void __launch_bounds__(kEnsMaxTile) ensemble_fixed_measure_kernel(const EnsCfg *__restrict__ cfgs,
                                                                           const EnsTile *__restrict__ tiles,
                                                                           int parity, double *partials)
{
    const EnsTile w = tiles[blockIdx.x];
    const EnsCfg c = cfgs[w.cfg];
    const uint32_t h0 = w.h0 + threadIdx.x / kEnsFixedLanes;
    const int lane = (int)(threadIdx.x % kEnsFixedLanes);
    const bool active = h0 < c.g.Vh;
    const uint32_t h = active ? h0 : c.g.Vh - 1;
    double f = 0.0, th = 0.0;
    const void *links = REC ? c.rec : c.field;
    if (c.fmt == FA) measure_site_fixed<FA, kEnsFixedLanes, 0, REC>(links, c.gf, c.g, parity, h, lane, active, f, th);
    else if (FB != FA && c.fmt == FB)
        measure_site_fixed<FB, kEnsFixedLanes, 0, REC>(links, c.gf, c.g, parity, h, lane, active, f, th);
    block_sum2_any(f, th, partials + 2 * blockIdx.x);
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

template <int FA, int FB, bool SR, bool NT>
static const void *sweep_symbol()
{
    return reinterpret_cast<const void *>(&ensemble_sweep_kernel<FA, FB, SR, NT>);
}

template <int FA, int FB>
static hipError_t launch_ens_sweep_t(const EnsLaunch &L, int parity, const EnsRelax &r, uint32_t sweep_offset,
                                     bool sr, bool nt, double *meas, hipStream_t s)
{
    const dim3 grid(L.grid), block(L.tile);
    if (meas) {
        // the fused measurement: overrelaxation with non-temporal access only
        if (sr || !nt) return hipErrorInvalidValue;
        hipLaunchKernelGGL((ensemble_sweep_kernel<FA, FB, false, true, true>), grid, block, 0, s, L.cfgs, L.tiles, L.n_tiles, L.sweep_base, parity, r, sweep_offset, meas);
    } else if (sr) {
        if (nt) hipLaunchKernelGGL((ensemble_sweep_kernel<FA, FB, true, true>), grid, block, 0, s, L.cfgs, L.tiles, L.n_tiles, L.sweep_base, parity, r, sweep_offset, nullptr);
        else hipLaunchKernelGGL((ensemble_sweep_kernel<FA, FB, true, false>), grid, block, 0, s, L.cfgs, L.tiles, L.n_tiles, L.sweep_base, parity, r, sweep_offset, nullptr);
    } else {
        if (nt) hipLaunchKernelGGL((ensemble_sweep_kernel<FA, FB, false, true>), grid, block, 0, s, L.cfgs, L.tiles, L.n_tiles, L.sweep_base, parity, r, sweep_offset, nullptr);
        else hipLaunchKernelGGL((ensemble_sweep_kernel<FA, FB, false, false>), grid, block, 0, s, L.cfgs, L.tiles, L.n_tiles, L.sweep_base, parity, r, sweep_offset, nullptr);
    }
    return hipGetLastError();
}

// format pairs with an instantiation: (a, b) with a <= b
#define LGF_ENS_PAIRS(X) X(0, 0) X(0, 1) X(0, 2) X(0, 3) X(1, 1) X(1, 2) X(1, 3) X(2, 2) X(2, 3) X(3, 3)

hipError_t launch_ensemble_sweep(int fa, int fb, const EnsLaunch &L, int parity, const EnsRelax &r,
                                 uint32_t sweep_offset, bool sr, bool nt, hipStream_t s, double *meas)
{
    if (fa > fb) { const int t = fa; fa = fb; fb = t; }
#define LGF_CASE(A, B) if (fa == A && fb == B) return launch_ens_sweep_t<A, B>(L, parity, r, sweep_offset, sr, nt, meas, s);
    LGF_ENS_PAIRS(LGF_CASE)
#undef LGF_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_ensemble_measure(int fa, int fb, const EnsLaunch &L, uint32_t n_tiles, int parity, bool reunit_fwd,
                                   bool reunit_bwd, double *partials, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    if (fa > fb) { const int t = fa; fa = fb; fb = t; }
    const int rf = reunit_fwd ? 1 : 0, rb = reunit_bwd ? 1 : 0;
#define LGF_CASE(A, B)                                                                                  \
    if (fa == A && fb == B) {                                                                           \
        hipLaunchKernelGGL((ensemble_measure_kernel<A, B>), dim3(n_tiles), dim3(L.tile), 0, s, L.cfgs,   \
                           L.tiles, parity, rf, rb, partials);                                         \
        return hipGetLastError();                                                                       \
    }
    LGF_ENS_PAIRS(LGF_CASE)
#undef LGF_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_ensemble_finish(const double *partials, uint32_t n_tiles, const EnsSpan *spans, uint32_t n_spans,
                                  double *out, hipStream_t s)
{
    if (n_spans == 0) return hipSuccess;
    hipLaunchKernelGGL(ensemble_finish_kernel, dim3(n_spans), dim3(256), 0, s, partials, n_tiles, spans, out);
    return hipGetLastError();
}

__global__ void set_u64_kernel(uint64_t *p, uint64_t v)
{
    if (threadIdx.x == 0) *p = v;
}

hipError_t launch_set_u64(uint64_t *p, uint64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

// format pairs of the fixed-link kernels: (a, b) with a <= b (4: FP64 on
// the split links, g in FP64-12)
#define LGF_ENS_FIXED_PAIRS(X) X(0, 0) X(2, 2) X(2, 3) X(3, 3) X(2, 4) X(4, 4)

bool ensemble_fixed_pair(int fa, int fb)
{
    if (fa > fb) { const int t = fa; fa = fb; fb = t; }
#define LGF_CASE(A, B) if (fa == A && fb == B) return true;
    LGF_ENS_FIXED_PAIRS(LGF_CASE)
#undef LGF_CASE
    return false;
}

// pairs whose formats both have per-site link records (the 12-real formats
// and the split links)
constexpr bool has_records(int f) { return f == kF32_12 || f == kF64_12 || f == kF64_12S; }
template <int FA, int FB>
constexpr bool kRecPair = has_records(FA) && has_records(FB);

bool ensemble_fixed_records_pair(int fa, int fb)
{
    return ensemble_fixed_pair(fa, fb) && has_records(fa) && has_records(fb);
}

template <int FA, int FB, bool REC>
static hipError_t launch_ens_fixed_r(const EnsLaunch &L, int parity, const EnsRelax &r, uint32_t sweep_offset,
                                     bool sr, int post, double *meas, hipStream_t s)
{
    const dim3 grid(L.grid), block(L.tile);
#define LGF_EF(SRV, P)                                                                                          \
    hipLaunchKernelGGL((ensemble_fixed_kernel<FA, FB, SRV, P, REC>), grid, block, 0, s, L.cfgs, L.tiles,         \
                       L.n_tiles, L.sweep_base, parity, r, sweep_offset, meas)
    if (post == 2 && !meas) return hipErrorInvalidValue;
    if (sr) {
        if (post == 0) LGF_EF(true, 0);
        else if (post == 1) LGF_EF(true, 1);
        else LGF_EF(true, 2);
    } else {
        if (post == 0) LGF_EF(false, 0);
        else if (post == 1) LGF_EF(false, 1);
        else LGF_EF(false, 2);
    }
#undef LGF_EF
    return hipGetLastError();
}

template <int FA, int FB>
static hipError_t launch_ens_fixed_t(const EnsLaunch &L, int parity, const EnsRelax &r, uint32_t sweep_offset,
                                     bool sr, int post, double *meas, hipStream_t s, bool rec)
{
    if (rec) {
        if constexpr (kRecPair<FA, FB>)
            return launch_ens_fixed_r<FA, FB, true>(L, parity, r, sweep_offset, sr, post, meas, s);
        else
            return hipErrorInvalidValue;
    }
    return launch_ens_fixed_r<FA, FB, false>(L, parity, r, sweep_offset, sr, post, meas, s);
}

hipError_t launch_ensemble_fixed_sweep(int fa, int fb, const EnsLaunch &L, int parity, const EnsRelax &r,
                                       uint32_t sweep_offset, bool sr, int post, double *meas, hipStream_t s,
                                       bool rec)
{
    if (post < 0 || post > 2 || L.tile % 64 != 0) return hipErrorInvalidValue;
    if (fa > fb) { const int t = fa; fa = fb; fb = t; }
#define LGF_CASE(A, B)                                                                                       \
    if (fa == A && fb == B) return launch_ens_fixed_t<A, B>(L, parity, r, sweep_offset, sr, post, meas, s, rec);
    LGF_ENS_FIXED_PAIRS(LGF_CASE)
#undef LGF_CASE
    return hipErrorInvalidValue;
}

template <int FA, int FB>
static hipError_t launch_ens_fixed_measure_t(const EnsLaunch &L, uint32_t n_tiles, int parity, double *partials,
                                             hipStream_t s, bool rec)
{
    if (rec) {
        if constexpr (kRecPair<FA, FB>)
            hipLaunchKernelGGL((ensemble_fixed_measure_kernel<FA, FB, true>), dim3(n_tiles), dim3(L.tile), 0, s,
                               L.cfgs, L.tiles, parity, partials);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((ensemble_fixed_measure_kernel<FA, FB, false>), dim3(n_tiles), dim3(L.tile), 0, s,
                           L.cfgs, L.tiles, parity, partials);
    }
    return hipGetLastError();
}

hipError_t launch_ensemble_fixed_measure(int fa, int fb, const EnsLaunch &L, uint32_t n_tiles, int parity,
                                         double *partials, hipStream_t s, bool rec)
{
    if (n_tiles == 0) return hipSuccess;
    if (fa > fb) { const int t = fa; fa = fb; fb = t; }
#define LGF_CASE(A, B) \
    if (fa == A && fb == B) return launch_ens_fixed_measure_t<A, B>(L, n_tiles, parity, partials, s, rec);
    LGF_ENS_FIXED_PAIRS(LGF_CASE)
#undef LGF_CASE
    return hipErrorInvalidValue;
}

template <int FA, int FB>
static const void *fixed_symbol(bool sr, bool rec)
{
    if constexpr (kRecPair<FA, FB>)
        if (rec)
            return sr ? reinterpret_cast<const void *>(&ensemble_fixed_kernel<FA, FB, true, 0, true>)
                      : reinterpret_cast<const void *>(&ensemble_fixed_kernel<FA, FB, false, 0, true>);
    return sr ? reinterpret_cast<const void *>(&ensemble_fixed_kernel<FA, FB, true, 0, false>)
              : reinterpret_cast<const void *>(&ensemble_fixed_kernel<FA, FB, false, 0, false>);
}

int ensemble_fixed_grid(int fa, int fb, bool sr, int tile, int grid_mult, bool rec)
{
    if (fa > fb) { const int t = fa; fa = fb; fb = t; }
    const void *fn = nullptr;
#define LGF_CASE(A, B) \
    if (fa == A && fb == B) fn = fixed_symbol<A, B>(sr, rec);
    LGF_ENS_FIXED_PAIRS(LGF_CASE)
#undef LGF_CASE
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, tile, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu * (grid_mult > 1 ? grid_mult : 1);
}

int ensemble_persistent_grid(int fa, int fb, bool sr, bool nt, int tile, int grid_mult)
{
    if (fa > fb) { const int t = fa; fa = fb; fb = t; }
    const void *fn = nullptr;
#define LGF_CASE(A, B)                                                                  \
    if (fa == A && fb == B)                                                             \
        fn = sr ? (nt ? sweep_symbol<A, B, true, true>() : sweep_symbol<A, B, true, false>()) \
                : (nt ? sweep_symbol<A, B, false, true>() : sweep_symbol<A, B, false, false>());
    LGF_ENS_PAIRS(LGF_CASE)
#undef LGF_CASE
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, tile, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu * (grid_mult > 1 ? grid_mult : 1);
}

}  // namespace lgf
