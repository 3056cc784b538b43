// lgf_kernels.hip -- gfx950 (CDNA4) kernels of the checkerboard SU(3) Landau
// gauge fixing of Schroeck and Vogt (arXiv:1305.3440): the relaxation sweep
// (Sec. 3, Eqs. (7)-(9), OR Sec. 3.1, SR Sec. 3.2), the F / theta reductions
// (Eqs. (2), (4), (5)) fused with FP64 reunitarization, format conversion,
// the seeded synthetic-field generator and canonical-array I/O.
//
// The sweep is bound by HBM bandwidth: a site update must read and write the
// 8 links that touch the site and does ~3k flops on them, far below the
// machine balance of either precision.  There is no dense contraction, so no
// MFMA; the design work is in the memory stream: a parity-split structure of
// arrays (lgf_device.hpp) so that every load and store of a wavefront is a
// contiguous 512 B - 1 KB run, all 8 links of a site held in registers
// between the gather and the store (no re-reads), and 1, 2 or 4 lanes per
// site to trade registers (occupancy) against redundant SU(2) arithmetic.
#include "lgf_device.hpp"
#include "lgf_internal.hpp"
#include "lgf_site.hpp"

namespace lgf {

size_t link_bytes(int format)
{
    switch (format) {
    case kF64_18: return 18 * sizeof(double);
    case kF32_18: return 18 * sizeof(float);
    case kF32_12: return 12 * sizeof(float);
    case kF64_12: return 12 * sizeof(double);
    default: return 0;
    }
}

// ----------------------------------------------------------------------------
// Relaxation sweep
// ----------------------------------------------------------------------------

// One half-sweep: the sites [h_begin, h_end) of one parity, LPS lanes per
// site, cut into n_tiles tiles of blockDim.x lanes.  Workgroup b takes the
// tiles b, b + n_groups, b + 2 n_groups, ... (spt of them at most), so the
// workgroups in flight always cover neighbouring tiles.  MEAS: the links are
// reunitarized as they are written and workgroup b leaves the sums of its
// sites' F and theta contributions in partials[2b], partials[2b + 1].
template <int F, int LPS, bool SR, bool NT, bool OOP, bool ACC, bool MEAS>
__global__ void __launch_bounds__(256) sweep_kernel(void *__restrict__ field, Geom g, int parity,
                                                     RelaxArgs<typename Fmt<F>::T> a, int xcd_remap,
                                                     uint32_t n_groups, uint32_t n_tiles, uint32_t spt,
                                                     uint32_t h_begin, uint32_t h_end,
                                                     void *__restrict__ out_field, double *__restrict__ partials)
{
    uint32_t b = blockIdx.x;
    if (xcd_remap) {
        // workgroups are dealt to the 8 XCDs round-robin; give XCD k the
        // contiguous range [k*per, (k+1)*per) of workgroups so that
        // neighbouring tiles share its L2
        const uint32_t per = gridDim.x >> 3;
        b = (b & 7u) * per + (b >> 3);
        if (b >= n_groups) return;  // the whole workgroup: no partials slot
    }
    MeasAcc acc;
    auto one_tile = [&](uint32_t tile) {
        // Vh <= 2^30 and LPS <= 4, so tile * blockDim + lane < 2^32
        const uint32_t tid = tile * blockDim.x + threadIdx.x;
        const uint32_t grp = h_begin + tid / LPS;
        const int lane = (int)(tid % LPS);
        const bool active = grp < h_end;
        update_site<F, LPS, SR, NT, 0, OOP, ACC, MEAS>(field, g, parity, active ? grp : h_end - 1, lane, active,
                                                       a, nullptr, out_field, &acc);
    };
    if (spt == 1) {
        one_tile(b);  // the common case without a loop around the register-heavy update
    } else {
        for (uint32_t k = 0; k < spt; ++k) {
            const uint32_t tile = b + k * n_groups;
            if (tile >= n_tiles) break;  // uniform over the workgroup
            one_tile(tile);
        }
    }
    if constexpr (MEAS) block_sum2_any(acc.f, acc.th, partials + 2 * b);
}

template <int F, int LPS, bool SR, bool NT, bool OOP, bool ACC, bool MEAS = false>
static void launch_sweep_kernel(dim3 grid, int block, hipStream_t s, void *field, const Geom &g, int parity,
                                const RelaxArgs<typename Fmt<F>::T> &ra, int xcd_remap, uint32_t n_groups,
                                uint32_t n_tiles, uint32_t spt, uint32_t h_begin, uint32_t h_end, void *out,
                                double *partials = nullptr)
{
    hipLaunchKernelGGL((sweep_kernel<F, LPS, SR, NT, OOP, ACC, MEAS>), grid, dim3(block), 0, s, field, g, parity,
                       ra, xcd_remap, n_groups, n_tiles, spt, h_begin, h_end, out, partials);
}

uint32_t sweep_groups(const Geom &g, const SweepTuning &t)
{
    const uint64_t threads = (uint64_t)g.Vh * (uint64_t)t.lanes_per_site;
    const uint32_t nb = (uint32_t)((threads + t.block - 1) / t.block);
    const uint32_t spt = (uint32_t)(t.sites_per_thread > 1 ? t.sites_per_thread : 1);
    return (nb + spt - 1) / spt;
}

template <int F, int LPS, bool NT, bool OOP>
static hipError_t launch_sweep_t(void *field, const Geom &g, const SweepArgs &a, const SweepTuning &t,
                                 hipStream_t s)
{
    if (OOP && (a.out == nullptr || a.out == field || a.h_end != 0)) return hipErrorInvalidValue;
    using T = typename Fmt<F>::T;
    const uint32_t h_begin = a.h_end ? a.h_begin : 0, h_end = a.h_end ? a.h_end : g.Vh;
    const uint64_t threads = (uint64_t)(h_end - h_begin) * LPS;
    const uint32_t nb = (uint32_t)((threads + t.block - 1) / t.block);          // tiles
    const uint32_t spt = (uint32_t)(t.sites_per_thread > 1 ? t.sites_per_thread : 1);
    const uint32_t ng = (nb + spt - 1) / spt;                                     // workgroups
    const uint32_t grid = t.xcd_remap ? ((ng + 7u) / 8u) * 8u : ng;
    RelaxArgs<T> ra{(T)a.omega, (a.omega != 1.0) ? 1 : 0, 0, (uint32_t)a.seed, (uint32_t)(a.seed >> 32),
                    (uint32_t)a.sweep_index, a.instance, a.gacc, a.sweep_base};
    const bool sr = a.p_sr > 0.0;
    if (sr) ra.sr_threshold = (uint64_t)floor(a.p_sr * 4294967296.0);
    if (a.meas) {
        // the fused reunitarize + measure: overrelaxation, non-temporal, whole half-sweeps
        if (sr || a.h_end != 0) return hipErrorInvalidValue;
        if constexpr (NT) {
            if (a.gacc) {
                if constexpr (F == kF32_12 || F == kF32_18)
                    launch_sweep_kernel<F, LPS, false, NT, OOP, true, true>(grid, t.block, s, field, g, a.parity,
                                                                            ra, t.xcd_remap, ng, nb, spt, h_begin,
                                                                            h_end, a.out, a.meas);
                else
                    return hipErrorInvalidValue;
            } else {
                launch_sweep_kernel<F, LPS, false, NT, OOP, false, true>(grid, t.block, s, field, g, a.parity, ra,
                                                                         t.xcd_remap, ng, nb, spt, h_begin, h_end,
                                                                         a.out, a.meas);
            }
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (a.gacc) {
        // the accumulated gauge transformation belongs to the FP32 bulk only
        if constexpr (F == kF32_12 || F == kF32_18) {
            if (sr)
                launch_sweep_kernel<F, LPS, true, NT, OOP, true>(grid, t.block, s, field, g, a.parity, ra,
                                                                 t.xcd_remap, ng, nb, spt, h_begin, h_end, a.out);
            else
                launch_sweep_kernel<F, LPS, false, NT, OOP, true>(grid, t.block, s, field, g, a.parity, ra,
                                                                  t.xcd_remap, ng, nb, spt, h_begin, h_end, a.out);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (sr) {
        launch_sweep_kernel<F, LPS, true, NT, OOP, false>(grid, t.block, s, field, g, a.parity, ra, t.xcd_remap,
                                                          ng, nb, spt, h_begin, h_end, a.out);
    } else {
        launch_sweep_kernel<F, LPS, false, NT, OOP, false>(grid, t.block, s, field, g, a.parity, ra, t.xcd_remap,
                                                           ng, nb, spt, h_begin, h_end, a.out);
    }
    return hipGetLastError();
}

template <int F>
static hipError_t launch_sweep_f(void *field, const Geom &g, const SweepArgs &a, const SweepTuning &t,
                                 hipStream_t s)
{
    // out of place only with non-temporal access (the variant that can use it)
    const bool oop = a.out != nullptr;
    if (oop && !t.nontemporal) return hipErrorInvalidValue;
    const int key = t.lanes_per_site * 2 + (t.nontemporal ? 1 : 0);
    switch (key) {
    case 2: return launch_sweep_t<F, 1, false, false>(field, g, a, t, s);
    case 3: return oop ? launch_sweep_t<F, 1, true, true>(field, g, a, t, s)
                       : launch_sweep_t<F, 1, true, false>(field, g, a, t, s);
    case 4: return launch_sweep_t<F, 2, false, false>(field, g, a, t, s);
    case 5: return oop ? launch_sweep_t<F, 2, true, true>(field, g, a, t, s)
                       : launch_sweep_t<F, 2, true, false>(field, g, a, t, s);
    case 8: return launch_sweep_t<F, 4, false, false>(field, g, a, t, s);
    case 9: return oop ? launch_sweep_t<F, 4, true, true>(field, g, a, t, s)
                       : launch_sweep_t<F, 4, true, false>(field, g, a, t, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(int format, void *field, const Geom &g, const SweepArgs &a,
                        const SweepTuning &t, hipStream_t s)
{
    if (t.block <= 0 || t.block > 256 || (t.block % 64) != 0) return hipErrorInvalidValue;
    switch (format) {
    case kF64_18: return launch_sweep_f<kF64_18>(field, g, a, t, s);
    case kF32_18: return launch_sweep_f<kF32_18>(field, g, a, t, s);
    case kF32_12: return launch_sweep_f<kF32_12>(field, g, a, t, s);
    case kF64_12: return launch_sweep_f<kF64_12>(field, g, a, t, s);
    default: return hipErrorInvalidValue;
    }
}

// ----------------------------------------------------------------------------
// F and theta: per-block partial sums, then one deterministic final sum.
// ----------------------------------------------------------------------------

template <int F>
__global__ void __launch_bounds__(kMeasureBlock) measure_kernel(void *__restrict__ field, Geom g,
                                                                int parity, int reunit_fwd,
                                                                int reunit_bwd, double *partials)
{
    const uint32_t h0 = blockIdx.x * kMeasureBlock + threadIdx.x;
    const bool active = h0 < g.Vh;
    double f, th;
    measure_site<F>(field, g, parity, active ? h0 : g.Vh - 1, active, reunit_fwd, reunit_bwd, f, th);
    block_sum2<kMeasureBlock>(f, th, partials + 2 * blockIdx.x);
}

int measure_blocks(const Geom &g) { return (int)((g.Vh + kMeasureBlock - 1) / kMeasureBlock); }

hipError_t launch_measure(int format, void *field, const Geom &g, int parity, bool reunit_fwd,
                          bool reunit_bwd, double *partials, int *n_partials, hipStream_t s)
{
    const int nb = measure_blocks(g);
    *n_partials = nb;
    const int rf = reunit_fwd ? 1 : 0, rb = reunit_bwd ? 1 : 0;
    switch (format) {
    case kF64_18: hipLaunchKernelGGL((measure_kernel<kF64_18>), dim3(nb), dim3(kMeasureBlock), 0, s, field, g, parity, rf, rb, partials); break;
    case kF32_18: hipLaunchKernelGGL((measure_kernel<kF32_18>), dim3(nb), dim3(kMeasureBlock), 0, s, field, g, parity, rf, rb, partials); break;
    case kF32_12: hipLaunchKernelGGL((measure_kernel<kF32_12>), dim3(nb), dim3(kMeasureBlock), 0, s, field, g, parity, rf, rb, partials); break;
    case kF64_12: hipLaunchKernelGGL((measure_kernel<kF64_12>), dim3(nb), dim3(kMeasureBlock), 0, s, field, g, parity, rf, rb, partials); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Deterministic final sum: thread t adds partials t, t+256, ... in order,
// then a fixed tree over the block.
// One workgroup reads every pair, so the sum is limited by the loads one CU
// keeps in flight: 1024 lanes with 8 independent 16-byte loads each.  Lane t
// adds pairs t + 1024 (8 j + k) into accumulator k, j = 0, 1, ...; the 8
// accumulators are then added in order k = 0..7 and the lanes in the fixed
// tree of block_sum2 -- a fixed order for a given n.
constexpr int kFinishBlock = 1024, kFinishAcc = 8;

__global__ void __launch_bounds__(kFinishBlock) finish_measure_kernel(const double *partials, int n, double V,
                                                                      double *out)
{
    const double2 *p = reinterpret_cast<const double2 *>(partials);
    double a[kFinishAcc], b[kFinishAcc];
#pragma unroll
    for (int k = 0; k < kFinishAcc; ++k) a[k] = b[k] = 0.0;
    const int step = kFinishBlock * kFinishAcc;
    int i = threadIdx.x;
    for (; i + (kFinishAcc - 1) * kFinishBlock < n; i += step) {
        double2 v[kFinishAcc];
#pragma unroll
        for (int k = 0; k < kFinishAcc; ++k) v[k] = p[i + k * kFinishBlock];
#pragma unroll
        for (int k = 0; k < kFinishAcc; ++k) {
            a[k] += v[k].x;
            b[k] += v[k].y;
        }
    }
    for (int k = 0; k < kFinishAcc && i + k * kFinishBlock < n; ++k) {
        const double2 v = p[i + k * kFinishBlock];
        a[k] += v.x;
        b[k] += v.y;
    }
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int k = 0; k < kFinishAcc; ++k) {
        ta += a[k];
        tb += b[k];
    }
    __shared__ double r[2];
    block_sum2<kFinishBlock>(ta, tb, r);
    if (threadIdx.x == 0) {
        out[0] = r[0] / (12.0 * V);
        out[1] = r[1] / (3.0 * V);
    }
}

hipError_t launch_finish_measure(const double *partials, int n, double V, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(finish_measure_kernel, dim3(1), dim3(kFinishBlock), 0, s, partials, n, V, out);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Format conversion / reunitarization (element-wise over all 4V links)
// ----------------------------------------------------------------------------

template <int FS, int FD>
__global__ void __launch_bounds__(256) convert_kernel(const void *__restrict__ src, void *__restrict__ dst,
                                                      uint32_t Vh, int reunit)
{
    const uint32_t h = blockIdx.x * 256 + threadIdx.x;
    if (h >= Vh) return;
    const int plane = blockIdx.y;  // parity*4 + mu
    mat3<typename Fmt<FS>::T> a;
    load_link<FS>(a, block_ptr<FS>(const_cast<void *>(src), Vh, plane >> 2, plane & 3), Vh, h);
    mat3<double> d;
    convert(d, a);
    if (reunit) reunitarize(d);
    mat3<typename Fmt<FD>::T> o;
    convert(o, d);
    store_link<FD>(block_ptr<FD>(dst, Vh, plane >> 2, plane & 3), Vh, h, o);
}

template <int FS>
static hipError_t launch_convert_s(const void *src, int fd, void *dst, uint32_t Vh, int reunit, hipStream_t s)
{
    const dim3 grid((Vh + 255) / 256, 8);
    switch (fd) {
    case kF64_18: hipLaunchKernelGGL((convert_kernel<FS, kF64_18>), grid, dim3(256), 0, s, src, dst, Vh, reunit); break;
    case kF32_18: hipLaunchKernelGGL((convert_kernel<FS, kF32_18>), grid, dim3(256), 0, s, src, dst, Vh, reunit); break;
    case kF32_12: hipLaunchKernelGGL((convert_kernel<FS, kF32_12>), grid, dim3(256), 0, s, src, dst, Vh, reunit); break;
    case kF64_12: hipLaunchKernelGGL((convert_kernel<FS, kF64_12>), grid, dim3(256), 0, s, src, dst, Vh, reunit); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_convert(int fs, const void *src, int fd, void *dst, const Geom &g, bool reunit,
                          hipStream_t s)
{
    const int r = reunit ? 1 : 0;
    switch (fs) {
    case kF64_18: return launch_convert_s<kF64_18>(src, fd, dst, g.Vh, r, s);
    case kF32_18: return launch_convert_s<kF32_18>(src, fd, dst, g.Vh, r, s);
    case kF32_12: return launch_convert_s<kF32_12>(src, fd, dst, g.Vh, r, s);
    case kF64_12: return launch_convert_s<kF64_12>(src, fd, dst, g.Vh, r, s);
    default: return hipErrorInvalidValue;
    }
}

// ----------------------------------------------------------------------------
// Seeded synthetic gauge field: U = exp(i eps sum_j a_j lambda_j), a_j normal,
// projected on SU(3), then U_mu(x) <- g(x) U_mu(x) g(x+mu)^dag with Haar g.
// ----------------------------------------------------------------------------

// four standard normals: Box-Muller on Philox words (0,1) and (2,3)
__device__ __forceinline__ void normals4(uint32_t k0, uint32_t k1, uint4 ctr, double n[4])
{
    const uint4 w = philox4x32_10(ctr, k0, k1);
    const double scale = 2.3283064365386963e-10;  // 2^-32
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double u1 = ((double)ws[2 * p] + 0.5) * scale;
        const double u2 = ((double)ws[2 * p + 1] + 0.5) * scale;
        const double r = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincos(6.283185307179586 * u2, &sn, &cs);
        n[2 * p] = r * cs;
        n[2 * p + 1] = r * sn;
    }
}

__device__ __forceinline__ void matmul(mat3<double> &r, const mat3<double> &a, const mat3<double> &b)
{
    left_mul<3>(r, a, b);
}

// exp(i eps H(a)) by scaling and squaring with a 16-term Taylor series
__device__ void su3_exp(mat3<double> &out, const double a[8], double eps)
{
    const double s3 = 0.57735026918962576;  // 1/sqrt(3)
    // X = i eps H with H = sum_j a_j lambda_j
    cpx<double> H[3][3];
    H[0][0] = {a[2] + a[7] * s3, 0.0};
    H[1][1] = {-a[2] + a[7] * s3, 0.0};
    H[2][2] = {-2.0 * a[7] * s3, 0.0};
    H[0][1] = {a[0], -a[1]};
    H[1][0] = {a[0], a[1]};
    H[0][2] = {a[3], -a[4]};
    H[2][0] = {a[3], a[4]};
    H[1][2] = {a[5], -a[6]};
    H[2][1] = {a[5], a[6]};
    mat3<double> X;
    double nrm = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            X.e[i][j] = {-eps * H[i][j].im, eps * H[i][j].re};
            nrm += norm2(X.e[i][j]);
        }
    nrm = sqrt(nrm);
    int k = 0;
    while (nrm >= 0.5 * ldexp(1.0, k)) ++k;
    const double sc = ldexp(1.0, -k);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) X.e[i][j] = {X.e[i][j].re * sc, X.e[i][j].im * sc};
    mat3<double> S, term, tmp;
    set_identity(S);
    set_identity(term);
    for (int n = 1; n <= 16; ++n) {
        matmul(tmp, term, X);
        const double inv = 1.0 / n;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                term.e[i][j] = {tmp.e[i][j].re * inv, tmp.e[i][j].im * inv};
                S.e[i][j] = S.e[i][j] + term.e[i][j];
            }
    }
    for (int q = 0; q < k; ++q) {
        matmul(tmp, S, S);
        S = tmp;
    }
    out = S;
}

// Haar SU(3): Ginibre matrix from 18 normals, Gram-Schmidt on the columns
// (positive real R diagonal), divided by the principal cube root of det.
__device__ void haar_su3(mat3<double> &g, uint32_t k0, uint32_t k1, uint32_t s)
{
    double n[20];
    for (int call = 0; call < 5; ++call) normals4(k0, k1, make_uint4(s, 0u, (uint32_t)call, 2u), n + 4 * call);
    const double r2 = 0.70710678118654752;
    mat3<double> Z;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Z.e[i][j] = {n[2 * (3 * i + j)] * r2, n[2 * (3 * i + j) + 1] * r2};
    for (int j = 0; j < 3; ++j) {
        cpx<double> v[3] = {Z.e[0][j], Z.e[1][j], Z.e[2][j]};
        for (int q = 0; q < j; ++q) {
            cpx<double> pr = {0.0, 0.0};
            for (int i = 0; i < 3; ++i) pr = pr + conj(g.e[i][q]) * v[i];
            for (int i = 0; i < 3; ++i) v[i] = v[i] - pr * g.e[i][q];
        }
        double nv = 0.0;
        for (int i = 0; i < 3; ++i) nv += norm2(v[i]);
        const double iv = 1.0 / sqrt(nv);
        for (int i = 0; i < 3; ++i) g.e[i][j] = {v[i].re * iv, v[i].im * iv};
    }
    const cpx<double> det =
        g.e[0][0] * (g.e[1][1] * g.e[2][2] - g.e[1][2] * g.e[2][1]) -
        g.e[0][1] * (g.e[1][0] * g.e[2][2] - g.e[1][2] * g.e[2][0]) +
        g.e[0][2] * (g.e[1][0] * g.e[2][1] - g.e[1][1] * g.e[2][0]);
    const double phi = atan2(det.im, det.re);
    double sn, cs;
    sincos(-phi / 3.0, &sn, &cs);
    const cpx<double> f = {cs, sn};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) g.e[i][j] = g.e[i][j] * f;
}

template <int F>
__global__ void __launch_bounds__(128) generate_kernel(void *__restrict__ field, Geom g, uint32_t k0,
                                                       uint32_t k1, double eps, int haar)
{
    const uint32_t s = blockIdx.x * 128 + threadIdx.x;
    if (s >= 2 * g.Vh) return;
    uint32_t r = s / g.L[3];
    const uint32_t x = s - r * g.L[3];
    const uint32_t row = r;
    const uint32_t y = r % g.L[2];
    r /= g.L[2];
    const uint32_t z = r % g.L[1];
    const uint32_t t = r / g.L[1];
    const int parity = (int)((t + z + y + x) & 1u);
    const uint32_t h = s >> 1;
    mat3<double> gx;
    if (haar) haar_su3(gx, k0, k1, s);
    for (int mu = 0; mu < 4; ++mu) {
        double a[8];
        normals4(k0, k1, make_uint4(s, (uint32_t)mu, 0u, 1u), a);
        normals4(k0, k1, make_uint4(s, (uint32_t)mu, 1u, 1u), a + 4);
        mat3<double> u;
        su3_exp(u, a, eps);
        reunitarize(u);
        if (haar) {
            // forward neighbour s + mu
            uint32_t sn;
            if (mu == 3) sn = row * g.L[3] + ((x + 1 == g.L[3]) ? 0 : x + 1);
            else {
                const uint32_t coord = (mu == 0) ? t : (mu == 1) ? z : y;
                const uint32_t stride = 2 * g.hs[mu];
                sn = (coord + 1 == g.L[mu]) ? s - (g.L[mu] - 1) * stride : s + stride;
            }
            mat3<double> gy, tmp;
            haar_su3(gy, k0, k1, sn);
            left_mul<3>(tmp, gx, u);
            right_mul_dag<3>(u, tmp, gy);
        }
        mat3<typename Fmt<F>::T> o;
        convert(o, u);
        store_link<F>(block_ptr<F>(field, g.Vh, parity, mu), g.Vh, h, o);
    }
}

hipError_t launch_generate(int format, void *field, const Geom &g, uint64_t seed, double eps, bool haar,
                           hipStream_t s)
{
    const uint32_t V = 2 * g.Vh;
    const dim3 grid((V + 127) / 128);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int hr = haar ? 1 : 0;
    switch (format) {
    case kF64_18: hipLaunchKernelGGL((generate_kernel<kF64_18>), grid, dim3(128), 0, s, field, g, k0, k1, eps, hr); break;
    case kF32_18: hipLaunchKernelGGL((generate_kernel<kF32_18>), grid, dim3(128), 0, s, field, g, k0, k1, eps, hr); break;
    case kF32_12: hipLaunchKernelGGL((generate_kernel<kF32_12>), grid, dim3(128), 0, s, field, g, k0, k1, eps, hr); break;
    case kF64_12: hipLaunchKernelGGL((generate_kernel<kF64_12>), grid, dim3(128), 0, s, field, g, k0, k1, eps, hr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Canonical double[site][mu][3][3][2] <-> private layout
// ----------------------------------------------------------------------------

__device__ __forceinline__ void lex_parity_half(const Geom &g, uint32_t s, int &parity, uint32_t &h)
{
    uint32_t r = s / g.L[3];
    const uint32_t x = s - r * g.L[3];
    const uint32_t y = r % g.L[2];
    r /= g.L[2];
    const uint32_t z = r % g.L[1];
    const uint32_t t = r / g.L[1];
    parity = (int)((t + z + y + x) & 1u);
    h = s >> 1;
}

template <int F>
__global__ void __launch_bounds__(256) canon_to_field_kernel(const double *__restrict__ canon, uint32_t s0,
                                                             uint32_t n, void *__restrict__ field, Geom g)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 4 * n) return;
    const uint32_t s = s0 + (i >> 2);
    const int mu = (int)(i & 3);
    int parity;
    uint32_t h;
    lex_parity_half(g, s, parity, h);
    const double *p = canon + (size_t)i * 18;
    mat3<typename Fmt<F>::T> u;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            u.e[a][b] = {(typename Fmt<F>::T)p[2 * (3 * a + b)], (typename Fmt<F>::T)p[2 * (3 * a + b) + 1]};
    store_link<F>(block_ptr<F>(field, g.Vh, parity, mu), g.Vh, h, u);
}

template <int F>
__global__ void __launch_bounds__(256) field_to_canon_kernel(const void *__restrict__ field,
                                                             const int64_t *__restrict__ sites, uint32_t s0,
                                                             uint32_t n, double *__restrict__ canon, Geom g)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 4 * n) return;
    const uint32_t s = sites ? (uint32_t)sites[i >> 2] : s0 + (i >> 2);
    const int mu = (int)(i & 3);
    int parity;
    uint32_t h;
    lex_parity_half(g, s, parity, h);
    mat3<typename Fmt<F>::T> u;
    load_link<F>(u, block_ptr<F>(const_cast<void *>(field), g.Vh, parity, mu), g.Vh, h);
    double *p = canon + (size_t)i * 18;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            p[2 * (3 * a + b)] = (double)u.e[a][b].re;
            p[2 * (3 * a + b) + 1] = (double)u.e[a][b].im;
        }
}

hipError_t launch_canon_to_field(int format, const double *canon, int64_t s0, int64_t n, void *field,
                                 const Geom &g, hipStream_t s)
{
    const dim3 grid((uint32_t)((4 * n + 255) / 256));
    const uint32_t a = (uint32_t)s0, b = (uint32_t)n;
    switch (format) {
    case kF64_18: hipLaunchKernelGGL((canon_to_field_kernel<kF64_18>), grid, dim3(256), 0, s, canon, a, b, field, g); break;
    case kF32_18: hipLaunchKernelGGL((canon_to_field_kernel<kF32_18>), grid, dim3(256), 0, s, canon, a, b, field, g); break;
    case kF32_12: hipLaunchKernelGGL((canon_to_field_kernel<kF32_12>), grid, dim3(256), 0, s, canon, a, b, field, g); break;
    case kF64_12: hipLaunchKernelGGL((canon_to_field_kernel<kF64_12>), grid, dim3(256), 0, s, canon, a, b, field, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_field_to_canon(int format, const void *field, const int64_t *sites, int64_t s0, int64_t n,
                                 double *canon, const Geom &g, hipStream_t s)
{
    const dim3 grid((uint32_t)((4 * n + 255) / 256));
    const uint32_t a = (uint32_t)s0, b = (uint32_t)n;
    switch (format) {
    case kF64_18: hipLaunchKernelGGL((field_to_canon_kernel<kF64_18>), grid, dim3(256), 0, s, field, sites, a, b, canon, g); break;
    case kF32_18: hipLaunchKernelGGL((field_to_canon_kernel<kF32_18>), grid, dim3(256), 0, s, field, sites, a, b, canon, g); break;
    case kF32_12: hipLaunchKernelGGL((field_to_canon_kernel<kF32_12>), grid, dim3(256), 0, s, field, sites, a, b, canon, g); break;
    case kF64_12: hipLaunchKernelGGL((field_to_canon_kernel<kF64_12>), grid, dim3(256), 0, s, field, sites, a, b, canon, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lgf

// ----------------------------------------------------------------------------
// Coulomb gauge: the functional of each timeslice holds its spatial links;
// the sweep updates all timeslices at once (4-D checkerboard, so the temporal
// links joining two timeslices are never written by two sites of a
// half-sweep), frozen timeslices are skipped, and F_C, theta_C are reduced
// per timeslice.
// ----------------------------------------------------------------------------

namespace lgf {

template <int F, bool SR, bool NT, bool ACC = false>
__global__ void __launch_bounds__(128) sweep_coulomb_kernel(void *__restrict__ field, Geom g, int parity,
                                                            RelaxArgs<typename Fmt<F>::T> a,
                                                            const uint8_t *__restrict__ slice_active)
{
    const uint32_t h0 = blockIdx.x * 128 + threadIdx.x;
    const bool active = h0 < g.Vh;
    update_site<F, 1, SR, NT, 1, false, ACC>(field, g, parity, active ? h0 : g.Vh - 1, 0, active, a, slice_active);
}

template <int F, bool NT>
static hipError_t launch_sweep_coulomb_t(void *field, const Geom &g, const SweepArgs &a,
                                         const uint8_t *slice_active, hipStream_t s)
{
    using T = typename Fmt<F>::T;
    const dim3 grid((g.Vh + 127) / 128);
    RelaxArgs<T> ra{(T)a.omega, (a.omega != 1.0) ? 1 : 0, 0, (uint32_t)a.seed, (uint32_t)(a.seed >> 32),
                    (uint32_t)a.sweep_index, a.instance, a.gacc, a.sweep_base};
    const bool sr = a.p_sr > 0.0;
    if (sr) ra.sr_threshold = (uint64_t)floor(a.p_sr * 4294967296.0);
    if (a.gacc) {
        // the accumulated gauge transformation belongs to the FP32 bulk only
        if constexpr (F == kF32_12 || F == kF32_18) {
            if (sr)
                hipLaunchKernelGGL((sweep_coulomb_kernel<F, true, NT, true>), grid, dim3(128), 0, s, field, g,
                                   a.parity, ra, slice_active);
            else
                hipLaunchKernelGGL((sweep_coulomb_kernel<F, false, NT, true>), grid, dim3(128), 0, s, field, g,
                                   a.parity, ra, slice_active);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (sr) {
        hipLaunchKernelGGL((sweep_coulomb_kernel<F, true, NT>), grid, dim3(128), 0, s, field, g, a.parity, ra,
                           slice_active);
    } else {
        hipLaunchKernelGGL((sweep_coulomb_kernel<F, false, NT>), grid, dim3(128), 0, s, field, g, a.parity, ra,
                           slice_active);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_coulomb(int format, void *field, const Geom &g, const SweepArgs &a,
                                const uint8_t *slice_active, bool nt, hipStream_t s)
{
    switch (format * 2 + (nt ? 1 : 0)) {
    case 0: return launch_sweep_coulomb_t<kF64_18, false>(field, g, a, slice_active, s);
    case 1: return launch_sweep_coulomb_t<kF64_18, true>(field, g, a, slice_active, s);
    case 2: return launch_sweep_coulomb_t<kF32_18, false>(field, g, a, slice_active, s);
    case 3: return launch_sweep_coulomb_t<kF32_18, true>(field, g, a, slice_active, s);
    case 4: return launch_sweep_coulomb_t<kF32_12, false>(field, g, a, slice_active, s);
    case 5: return launch_sweep_coulomb_t<kF32_12, true>(field, g, a, slice_active, s);
    case 6: return launch_sweep_coulomb_t<kF64_12, false>(field, g, a, slice_active, s);
    case 7: return launch_sweep_coulomb_t<kF64_12, true>(field, g, a, slice_active, s);
    default: return hipErrorInvalidValue;
    }
}

// grid (blocks per timeslice, Lt): every workgroup lies in one timeslice
template <int F>
__global__ void __launch_bounds__(kMeasureBlock) measure_coulomb_kernel(void *__restrict__ field, Geom g,
                                                                        int parity, int reunit_fwd,
                                                                        int reunit_bwd, double *partials)
{
    const uint32_t t = blockIdx.y;
    const uint32_t i = blockIdx.x * kMeasureBlock + threadIdx.x;
    const bool active = i < g.hs[0];
    const uint32_t h = t * g.hs[0] + (active ? i : g.hs[0] - 1);
    double f, th;
    measure_site<F, 1>(field, g, parity, h, active, reunit_fwd, reunit_bwd, f, th);
    block_sum2<kMeasureBlock>(f, th, partials + 2 * ((size_t)t * gridDim.x + blockIdx.x));
}

int coulomb_blocks_per_slice(const Geom &g) { return (int)((g.hs[0] + kMeasureBlock - 1) / kMeasureBlock); }

hipError_t launch_measure_coulomb(int format, void *field, const Geom &g, int parity, bool reunit_fwd,
                                  bool reunit_bwd, double *partials, hipStream_t s)
{
    const dim3 grid(coulomb_blocks_per_slice(g), g.L[0]);
    const int rf = reunit_fwd ? 1 : 0, rb = reunit_bwd ? 1 : 0;
    switch (format) {
    case kF64_18: hipLaunchKernelGGL((measure_coulomb_kernel<kF64_18>), grid, dim3(kMeasureBlock), 0, s, field, g, parity, rf, rb, partials); break;
    case kF32_18: hipLaunchKernelGGL((measure_coulomb_kernel<kF32_18>), grid, dim3(kMeasureBlock), 0, s, field, g, parity, rf, rb, partials); break;
    case kF32_12: hipLaunchKernelGGL((measure_coulomb_kernel<kF32_12>), grid, dim3(kMeasureBlock), 0, s, field, g, parity, rf, rb, partials); break;
    case kF64_12: hipLaunchKernelGGL((measure_coulomb_kernel<kF64_12>), grid, dim3(kMeasureBlock), 0, s, field, g, parity, rf, rb, partials); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// one workgroup per timeslice: both parity passes' partials in a fixed order;
// out[2t] = F_C(t), out[2t+1] = theta_C(t)
__global__ void __launch_bounds__(256) finish_coulomb_kernel(const double *__restrict__ partials, int bps,
                                                             double V3, double *__restrict__ out)
{
    const uint32_t t = blockIdx.x, Lt = gridDim.x;
    double a = 0.0, b = 0.0;
    for (uint32_t pass = 0; pass < 2; ++pass)
        for (int i = threadIdx.x; i < bps; i += 256) {
            const double *p = partials + 2 * (((size_t)pass * Lt + t) * bps + i);
            a += p[0];
            b += p[1];
        }
    __shared__ double r[2];
    block_sum2<256>(a, b, r);
    if (threadIdx.x == 0) {
        out[2 * t] = r[0] / (9.0 * V3);
        out[2 * t + 1] = r[1] / (3.0 * V3);
    }
}

hipError_t launch_finish_coulomb(const double *partials, const Geom &g, int bps, double *out, hipStream_t s)
{
    const double V3 = 2.0 * (double)g.hs[0];
    hipLaunchKernelGGL(finish_coulomb_kernel, dim3(g.L[0]), dim3(256), 0, s, partials,
                       bps, V3, out);
    return hipGetLastError();
}

}  // namespace lgf

// ----------------------------------------------------------------------------
// Plaquette: (1/(18 V)) sum_x sum_{mu<nu} Re tr[U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag
// U_nu(x)^dag], a gauge-invariant observable used to watch the gauge orbit.
// ----------------------------------------------------------------------------

namespace lgf {

template <int F>
__global__ void __launch_bounds__(kMeasureBlock) plaquette_kernel(void *__restrict__ field, Geom g,
                                                                  double *partials)
{
    using T = typename Fmt<F>::T;
    const int parity = blockIdx.y;
    const uint32_t h0 = blockIdx.x * kMeasureBlock + threadIdx.x;
    const bool active = h0 < g.Vh;
    const uint32_t h = active ? h0 : g.Vh - 1;
    const Site c = decode(g, parity, h);
    double sum = 0.0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            mat3<T> a, b, cc, d;
            load_link<F>(a, block_ptr<F>(field, g.Vh, parity, mu), g.Vh, h);
            load_link<F>(b, block_ptr<F>(field, g.Vh, parity ^ 1, nu), g.Vh, fwd_half(g, c, h, mu));
            load_link<F>(cc, block_ptr<F>(field, g.Vh, parity ^ 1, mu), g.Vh, fwd_half(g, c, h, nu));
            load_link<F>(d, block_ptr<F>(field, g.Vh, parity, nu), g.Vh, h);
            mat3<double> A, B, C, D, AB, CD;
            convert(A, a);
            convert(B, b);
            convert(C, cc);
            convert(D, d);
            left_mul<3>(AB, A, B);     // U_mu(x) U_nu(x+mu)
            left_mul<3>(CD, D, C);     // U_nu(x) U_mu(x+nu); the loop is AB (CD)^dag
            // Re tr[AB CD^dag] = sum_ij Re(AB_ij conj(CD_ij))
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    sum += AB.e[i][j].re * CD.e[i][j].re + AB.e[i][j].im * CD.e[i][j].im;
        }
    if (!active) sum = 0.0;
    block_sum2<kMeasureBlock>(sum, 0.0, partials + 2 * ((size_t)parity * gridDim.x + blockIdx.x));
}

hipError_t launch_plaquette(int format, void *field, const Geom &g, double *partials, int *n_partials,
                            hipStream_t s)
{
    const dim3 grid(measure_blocks(g), 2);
    *n_partials = 2 * (int)grid.x;
    switch (format) {
    case kF64_18: hipLaunchKernelGGL((plaquette_kernel<kF64_18>), grid, dim3(kMeasureBlock), 0, s, field, g, partials); break;
    case kF32_18: hipLaunchKernelGGL((plaquette_kernel<kF32_18>), grid, dim3(kMeasureBlock), 0, s, field, g, partials); break;
    case kF32_12: hipLaunchKernelGGL((plaquette_kernel<kF32_12>), grid, dim3(kMeasureBlock), 0, s, field, g, partials); break;
    case kF64_12: hipLaunchKernelGGL((plaquette_kernel<kF64_12>), grid, dim3(kMeasureBlock), 0, s, field, g, partials); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lgf

// ----------------------------------------------------------------------------
// Accumulated gauge transformation (mixed precision without orbit drift): the
// FP32 bulk multiplies every site's G into g(x); at the switch the FP64 links
// are rebuilt from the untouched FP64 input as g(x) U_mu(x) g(x+mu)^dag with
// g projected on SU(3) in FP64, an exact gauge transformation (Eq. (3)).
// ----------------------------------------------------------------------------

namespace lgf {

template <int F>
__global__ void __launch_bounds__(256) site_field_kernel(void *__restrict__ gf, uint32_t Vh, int mode)
{
    const uint32_t h = blockIdx.x * 256 + threadIdx.x;
    if (h >= Vh) return;
    const int parity = blockIdx.y;
    typename Fmt<F>::V *p = site_field_ptr<F>(gf, Vh, parity);
    mat3<typename Fmt<F>::T> o;
    if (mode == 0) {
        set_identity(o);
    } else {  // reunitarize in FP64
        mat3<typename Fmt<F>::T> u;
        load_link<F>(u, p, Vh, h);
        mat3<double> d;
        convert(d, u);
        reunitarize(d);
        convert(o, d);
    }
    store_link<F>(p, Vh, h, o);
}

hipError_t launch_site_field(int format, void *gf, const Geom &g, int mode, hipStream_t s)
{
    const dim3 grid((g.Vh + 255) / 256, 2);
    switch (format) {
    case kF64_18: hipLaunchKernelGGL((site_field_kernel<kF64_18>), grid, dim3(256), 0, s, gf, g.Vh, mode); break;
    case kF32_18: hipLaunchKernelGGL((site_field_kernel<kF32_18>), grid, dim3(256), 0, s, gf, g.Vh, mode); break;
    case kF32_12: hipLaunchKernelGGL((site_field_kernel<kF32_12>), grid, dim3(256), 0, s, gf, g.Vh, mode); break;
    case kF64_12: hipLaunchKernelGGL((site_field_kernel<kF64_12>), grid, dim3(256), 0, s, gf, g.Vh, mode); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// dst (format FD) <- g(x) src_mu(x) g(x+mu)^dag, src in format FS, g in FG;
// element-wise per link, so dst may be src when FD == FS
template <int FS, int FG, int FD>
__global__ void __launch_bounds__(256) gauge_transform_kernel(const void *src,
                                                              const void *__restrict__ gf, void *dst, Geom g)
{
    const uint32_t h = blockIdx.x * 256 + threadIdx.x;
    if (h >= g.Vh) return;
    const int parity = blockIdx.y >> 2, mu = blockIdx.y & 3;
    const Site c = decode(g, parity, h);
    mat3<typename Fmt<FS>::T> u;
    mat3<typename Fmt<FG>::T> gx, gy;
    load_link<FS>(u, block_ptr<FS>(const_cast<void *>(src), g.Vh, parity, mu), g.Vh, h);
    load_link<FG>(gx, site_field_ptr<FG>(const_cast<void *>(gf), g.Vh, parity), g.Vh, h);
    load_link<FG>(gy, site_field_ptr<FG>(const_cast<void *>(gf), g.Vh, parity ^ 1), g.Vh, fwd_half(g, c, h, mu));
    mat3<double> U, X, Y, t, r;
    convert(U, u);
    convert(X, gx);
    convert(Y, gy);
    reunitarize(X);
    reunitarize(Y);
    left_mul<3>(t, X, U);
    right_mul_dag<3>(r, t, Y);
    mat3<typename Fmt<FD>::T> o;
    convert(o, r);
    store_link<FD>(block_ptr<FD>(dst, g.Vh, parity, mu), g.Vh, h, o);
}

template <int FS, int FG>
static hipError_t launch_gt_d(int fd, const void *src, const void *gf, void *dst, const Geom &g, hipStream_t s)
{
    const dim3 grid((g.Vh + 255) / 256, 8);
    switch (fd) {
    case kF64_18: hipLaunchKernelGGL((gauge_transform_kernel<FS, FG, kF64_18>), grid, dim3(256), 0, s, src, gf, dst, g); break;
    case kF64_12: hipLaunchKernelGGL((gauge_transform_kernel<FS, FG, kF64_12>), grid, dim3(256), 0, s, src, gf, dst, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gauge_transform(int fs, const void *src, int fg, const void *gf, int fd, void *dst, const Geom &g,
                                  hipStream_t s)
{
#define LGF_GT_CASE(FS, FG) \
    if (fs == FS && fg == FG) return launch_gt_d<FS, FG>(fd, src, gf, dst, g, s);
    LGF_GT_CASE(kF64_18, kF32_12) LGF_GT_CASE(kF64_18, kF32_18) LGF_GT_CASE(kF64_18, kF64_12)
    LGF_GT_CASE(kF64_18, kF64_18) LGF_GT_CASE(kF64_12, kF32_12) LGF_GT_CASE(kF64_12, kF32_18)
    LGF_GT_CASE(kF64_12, kF64_12) LGF_GT_CASE(kF64_12, kF64_18)
#undef LGF_GT_CASE
    return hipErrorInvalidValue;
}

}  // namespace lgf
