// lgf_anneal.hip -- simulated annealing on gfx950: the heat-bath half-sweep.
//
// The paper lists simulated annealing among the methods its code supports
// (Sec. 1) and leaves the details to a reference.  The reading implemented
// here: the site update of Sec. 3 with the SU(2) step of every
// Cabibbo-Marinari subgroup replaced by a heat-bath draw at temperature T.
// With a the quaternion projection of the subgroup block w of W = G K and b
// the maximum of Eq. (9), the local functional on the subgroup is
// Re tr[s(r) w] = 2|a| <r, b>; r = x b is drawn with weight
// exp(2|a| <r, b> / T) against the Haar measure of SU(2): x0 with density
// sqrt(1 - x0^2) exp(alpha x0), alpha = 2|a|/T (Kennedy-Pendleton above
// alpha = 0.7, a uniform proposal below it, both accepting at least 40 % of
// their trials, at most 64 trials), (x1, x2, x3) uniform on the sphere of
// radius sqrt(1 - x0^2).  Random words: Philox4x32-10 keyed by the seed,
// counter (lexicographic site, sweep, instance, (k + 1) << 16 | trial) for
// subgroup k, trial 0xFFFF for the direction.
//
// The heat-bath arithmetic is FP64 and the kernel is instantiated for the FP64
// storage formats only: its accept-reject decisions must be the ones an FP64
// computation takes.  Like the relaxation sweep the update reads and writes
// the 8 links of a site once (HBM bound for the links; the transcendental
// functions of 1-2 trials per subgroup add ~20 % arithmetic).  The heat bath
// is the arithmetic of a whole site, so every lane that shares a site repeats
// it: on FP64-12 links one lane holds all 8 links of its site (96 VGPRs of
// rows 0 and 1; the kernel runs one wave per SIMD with part of its state in
// the accumulation registers) and the heat bath is paid once per site, 1.4-1.5x
// faster than two lanes per site; the 8 FP64-18 links do not fit one lane, so
// that format keeps two lanes per site, each holding two directions.
#include <type_traits>

#include "lgf_device.hpp"
#include "lgf_internal.hpp"
#include "lgf_site.hpp"

namespace lgf {

namespace {

constexpr uint32_t kSaTrials = 64;
constexpr double kSaSwitch = 0.7;
constexpr double kTwoPi = 2.0 * 3.14159265358979323846;

__device__ __forceinline__ double unit_uniform(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

__device__ __forceinline__ uint32_t sa_tag(int k, uint32_t t) { return ((uint32_t)(k + 1) << 16) | t; }

struct SaKey {
    uint32_t site, sweep, instance, k0, k1;
};

// x0 with density sqrt(1 - x0^2) exp(alpha x0) on [-1, 1]; returns the trials
// used (kSaTrials + 1 and x0 = 1 when none was accepted)
__device__ __forceinline__ uint32_t heatbath_x0(double alpha, const SaKey &key, int k, double &x0)
{
    for (uint32_t t = 0; t < kSaTrials; ++t) {
        const uint4 w = philox4x32_10(make_uint4(key.site, key.sweep, key.instance, sa_tag(k, t)), key.k0, key.k1);
        const double u1 = unit_uniform(w.x), u2 = unit_uniform(w.y);
        if (alpha >= kSaSwitch) {
            // lambda^2 = l ~ Gamma(3/2, rate 2 alpha), accepted with
            // probability sqrt(1 - l); x0 = 1 - 2 l
            const double u3 = unit_uniform(w.z), u4 = unit_uniform(w.w);
            const double c = cos(kTwoPi * u2);
            const double l = -(log(u1) + c * c * log(u3)) / (2.0 * alpha);
            if (u4 * u4 <= 1.0 - l) {
                x0 = 1.0 - 2.0 * l;
                return t + 1;
            }
        } else {
            const double x = 2.0 * u1 - 1.0;
            if (u2 * u2 <= (1.0 - x * x) * exp(2.0 * alpha * (x - 1.0))) {
                x0 = x;
                return t + 1;
            }
        }
    }
    x0 = 1.0;
    return kSaTrials + 1;
}

// The heat-bath step of subgroup K_IDX = (I, J) on W = G K at temperature T:
// W <- R W (when UPDATE_W), G <- R G; returns the trials used.
template <int I, int J, int K_IDX, bool UPDATE_W>
__device__ __forceinline__ uint32_t heatbath_step(mat3<double> &W, mat3<double> &G, double temp, const SaKey &key)
{
    const double a0 = 0.5 * (W.e[I][I].re + W.e[J][J].re);
    const double a3 = 0.5 * (W.e[I][I].im - W.e[J][J].im);
    const double a1 = 0.5 * (W.e[I][J].im + W.e[J][I].im);
    const double a2 = 0.5 * (W.e[I][J].re - W.e[J][I].re);
    const double na = sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3);
    double b0 = 1.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    if (na > 0.0) {
        b0 = a0 / na;
        b1 = -a1 / na;
        b2 = -a2 / na;
        b3 = -a3 / na;
    }
    double x0;
    const uint32_t trials = heatbath_x0(2.0 * na / temp, key, K_IDX, x0);
    const uint4 v = philox4x32_10(make_uint4(key.site, key.sweep, key.instance, sa_tag(K_IDX, 0xFFFFu)), key.k0,
                                  key.k1);
    const double ct = 2.0 * unit_uniform(v.x) - 1.0;
    const double phi = kTwoPi * unit_uniform(v.y);
    const double st = sqrt(1.0 - ct * ct);
    const double rad = sqrt(fmax(0.0, 1.0 - x0 * x0));
    const double x1 = rad * st * cos(phi), x2 = rad * st * sin(phi), x3 = rad * ct;
    // r = x b as quaternions: s(r) = s(x) s(b)
    const double r0 = x0 * b0 - (x1 * b1 + x2 * b2 + x3 * b3);
    const double r1 = x0 * b1 + b0 * x1 - (x2 * b3 - x3 * b2);
    const double r2 = x0 * b2 + b0 * x2 - (x3 * b1 - x1 * b3);
    const double r3 = x0 * b3 + b0 * x3 - (x1 * b2 - x2 * b1);
    // s(r) = [[r0 + i r3, r2 + i r1], [-r2 + i r1, r0 - i r3]]
    const cpx<double> s00 = {r0, r3}, s01 = {r2, r1}, s10 = {-r2, r1}, s11 = {r0, -r3};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<double> gi = G.e[I][c], gj = G.e[J][c];
        G.e[I][c] = s00 * gi + s01 * gj;
        G.e[J][c] = s10 * gi + s11 * gj;
        if constexpr (UPDATE_W) {
            const cpx<double> wi = W.e[I][c], wj = W.e[J][c];
            W.e[I][c] = s00 * wi + s01 * wj;
            W.e[J][c] = s10 * wi + s11 * wj;
        }
    }
    return trials;
}

// lanes per site: 1 on FP64-12 links, 2 on FP64-18 links
template <int F> constexpr int sa_lanes() { return F == kF64_12 ? 1 : 2; }
constexpr int kSaBlock = 128;  // lanes per workgroup

// One annealing half-sweep over the sites of one parity, LANES lanes per site
// (lane l gathers and stores directions l, l + LANES, ...).  With two lanes
// both run the same heat-bath steps on the same K and the same random words,
// so they hold the same G.  trials (may be NULL) accumulates the
// accept-reject trials of the launch: a wave sum, then one 64-bit atomic add
// per wave.
template <int F>
__global__ void __launch_bounds__(kSaBlock) anneal_kernel(void *__restrict__ field, Geom g, int parity, double temp,
                                                          uint32_t sweep, uint32_t instance, uint32_t k0, uint32_t k1,
                                                          unsigned long long *__restrict__ trials)
{
    static_assert(std::is_same<typename Fmt<F>::T, double>::value, "the heat bath runs on FP64 links");
    using S = Fmt<F>;
    constexpr int LANES = sa_lanes<F>();
    constexpr int NL = 4 / LANES;
    // Vh <= 2^30, so blockIdx * blockDim + lane < 2^32
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t grp = tid / LANES;
    const int lane = (int)(tid % LANES);
    const bool active = grp < g.Vh;
    const uint32_t h = active ? grp : g.Vh - 1;
    const Site c = decode(g, parity, h);

    mat3<double> uf[NL], ub[NL];
    uint32_t hb[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int mu = lane + k * LANES;
        hb[k] = back_half(g, c, h, mu);
        load_link<F, true>(uf[k], block_ptr<F>(field, g.Vh, parity, mu), g.Vh, h);
        load_link<F, true>(ub[k], block_ptr<F>(field, g.Vh, parity ^ 1, mu), g.Vh, hb[k]);
    }
    mat3<double> K;
    set_zero(K);
#pragma unroll
    for (int k = 0; k < NL; ++k) add_fwd_bwd(K, uf[k], ub[k]);
    if constexpr (LANES == 2) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                K.e[i][j].re += shfl_xor_t(K.e[i][j].re, 1);
                K.e[i][j].im += shfl_xor_t(K.e[i][j].im, 1);
            }
    }

    const SaKey key{lex_index(g, c), sweep, instance, k0, k1};
    mat3<double> G;
    set_identity(G);
    uint32_t n = heatbath_step<0, 1, 0, true>(K, G, temp, key);
    n += heatbath_step<0, 2, 1, true>(K, G, temp, key);
    n += heatbath_step<1, 2, 2, false>(K, G, temp, key);

    if (active) {
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int mu = lane + k * LANES;
            mat3<double> r, rb;
            left_mul<S::R>(r, G, uf[k]);
            right_mul_dag<S::R>(rb, ub[k], G);
            store_link<F, true>(block_ptr<F>(field, g.Vh, parity, mu), g.Vh, h, r);
            store_link<F, true>(block_ptr<F>(field, g.Vh, parity ^ 1, mu), g.Vh, hb[k], rb);
        }
    }
    if (trials) {
        uint32_t cnt = (active && lane == 0) ? n : 0u;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) cnt += __shfl_xor(cnt, m);
        if ((threadIdx.x & 63u) == 0 && cnt) atomicAdd(trials, (unsigned long long)cnt);
    }
}

template <int F>
hipError_t launch_anneal_f(void *field, const Geom &g, int parity, double temp, uint64_t seed, uint64_t sweep,
                           uint32_t instance, unsigned long long *trials, hipStream_t s)
{
    const uint64_t threads = (uint64_t)g.Vh * sa_lanes<F>();
    const uint32_t nb = (uint32_t)((threads + kSaBlock - 1) / kSaBlock);
    hipLaunchKernelGGL((anneal_kernel<F>), dim3(nb), dim3(kSaBlock), 0, s, field, g, parity, temp, (uint32_t)sweep,
                       instance, (uint32_t)seed, (uint32_t)(seed >> 32), trials);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_anneal(int format, void *field, const Geom &g, int parity, double temp, uint64_t seed,
                         uint64_t sweep, uint32_t instance, unsigned long long *trials, hipStream_t s)
{
    if (!(temp > 0.0)) return hipErrorInvalidValue;
    switch (format) {
    case kF64_18: return launch_anneal_f<kF64_18>(field, g, parity, temp, seed, sweep, instance, trials, s);
    case kF64_12: return launch_anneal_f<kF64_12>(field, g, parity, temp, seed, sweep, instance, trials, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lgf
