// lgf_site.hpp -- the per-site work of the relaxation sweep and of the
// F / theta measurement, shared by the single-lattice kernels and the
// persistent ensemble kernels.
#pragma once

#include "lgf_device.hpp"

namespace lgf {

// One Cabibbo-Marinari SU(2) step on rows/columns (I, J) of W = G K.
// Quaternion projection a of the 2x2 block (a scaled by 2, which the
// normalisation removes); maximum of Re tr[s(b) w] at b = (a0, -a)/|a|
// (Eq. (9)); OR: N[(1 - omega) + omega b] (first-order b^omega, Sec. 3.1);
// SR: b^2 (Sec. 3.2).  Then W <- R W and G <- R G on rows I, J.
template <int I, int J, bool UPDATE_W, typename T>
__device__ __forceinline__ void su2_step(mat3<T> &W, mat3<T> &G, T omega, bool overrelax, bool square)
{
    const T a0 = W.e[I][I].re + W.e[J][J].re;
    const T a3 = W.e[I][I].im - W.e[J][J].im;
    const T a1 = W.e[I][J].im + W.e[J][I].im;
    const T a2 = W.e[I][J].re - W.e[J][I].re;
    const T n2 = a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
    T r0 = T(1), r1 = T(0), r2 = T(0), r3 = T(0);
    if (n2 > T(0)) {
        const T inv = exact_rsqrt<T>(n2);
        const T b0 = a0 * inv, b1 = -a1 * inv, b2 = -a2 * inv, b3 = -a3 * inv;
        if (square) {
            r0 = b0 * b0 - (b1 * b1 + b2 * b2 + b3 * b3);
            r1 = T(2) * b0 * b1;
            r2 = T(2) * b0 * b2;
            r3 = T(2) * b0 * b3;
        } else if (overrelax) {
            const T c0 = (T(1) - omega) + omega * b0;
            const T c1 = omega * b1, c2 = omega * b2, c3 = omega * b3;
            const T ic = exact_rsqrt<T>(c0 * c0 + c1 * c1 + c2 * c2 + c3 * c3);
            r0 = c0 * ic; r1 = c1 * ic; r2 = c2 * ic; r3 = c3 * ic;
        } else {
            r0 = b0; r1 = b1; r2 = b2; r3 = b3;
        }
    }
    // s(r) = [[r0 + i r3, r2 + i r1], [-r2 + i r1, r0 - i r3]]
    const cpx<T> s00 = {r0, r3}, s01 = {r2, r1}, s10 = {-r2, r1}, s11 = {r0, -r3};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<T> gi = G.e[I][c], gj = G.e[J][c];
        G.e[I][c] = s00 * gi + s01 * gj;
        G.e[J][c] = s10 * gi + s11 * gj;
        if constexpr (UPDATE_W) {
            const cpx<T> wi = W.e[I][c], wj = W.e[J][c];
            W.e[I][c] = s00 * wi + s01 * wj;
            W.e[J][c] = s10 * wi + s11 * wj;
        }
    }
}


template <typename T> __device__ __forceinline__ T shfl_xor_t(T v, int m) { return __shfl_xor(v, m); }

// u <- u as stored in format F and read back; o receives the stored value
template <int F>
__device__ __forceinline__ void round_to_format(mat3<double> &u, mat3<typename Fmt<F>::T> &o)
{
    convert(o, u);
    if constexpr (Fmt<F>::R == 2) rebuild_row2(o);
    convert(u, o);
}

// |[(K - K^dag)/(2i)]_traceless|^2 = tr[Delta Delta^dag] of one site
__device__ __forceinline__ double theta_of_K(const mat3<double> &K)
{
    const double d0 = K.e[0][0].im, d1 = K.e[1][1].im, d2 = K.e[2][2].im;
    const double tr3 = (d0 + d1 + d2) * (1.0 / 3.0);
    double th = (d0 - tr3) * (d0 - tr3) + (d1 - tr3) * (d1 - tr3) + (d2 - tr3) * (d2 - tr3);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            // entries (i,j) and (j,i) have equal modulus |K_ij - conj(K_ji)| / 2
            const cpx<double> z = K.e[i][j] - conj(K.e[j][i]);
            th += 0.5 * norm2(z);
        }
    return th;
}

// Per-thread sums of the measurement fused into a half-sweep
struct MeasAcc {
    double f = 0.0;   // sum of Re tr of the forward links written
    double th = 0.0;  // sum of tr[Delta Delta^dag] of the sites updated
};

// Parameters of one relaxation half-sweep as the kernels see them.
template <typename T> struct RelaxArgs {
    T omega;
    int overrelax;          // omega != 1
    uint64_t sr_threshold;  // floor(p 2^32); only read when SR
    uint32_t key0, key1;    // Philox key (seed)
    uint32_t sweep, instance;
    void *gacc = nullptr;   // accumulated gauge transformation (site field) or none
    // when set, the stochastic-relaxation counter is *sweep_base + sweep (read
    // on the device, so a captured chunk replays for any starting counter)
    const uint64_t *sweep_base = nullptr;
};

// A site field (one SU(3) matrix per site, e.g. an accumulated gauge
// transformation) in the same parity-split layout as one direction of a link
// field: vector index = (parity*NV + slot)*Vh + h.
template <int F>
__device__ __forceinline__ typename Fmt<F>::V *site_field_ptr(void *field, uint32_t Vh, int parity)
{
    return reinterpret_cast<typename Fmt<F>::V *>(field) + (size_t)(parity * Fmt<F>::NV) * Vh;
}

// The local update of site h (half index) of the given parity by LPS lanes
// (lane in [0, LPS)): gather U_mu(x), U_mu(x - mu) for the lane's directions,
// K(x) = sum_mu U_mu(x) + U_mu(x - mu)^dag (Eq. (8) with the neighbours' g
// already applied), reduced over the LPS lanes; the three Cabibbo-Marinari
// SU(2) steps (0,1), (0,2), (1,2) accumulate G; store G U_mu(x) and
// U_mu(x - mu) G^dag.  Inactive lanes compute on a valid site and store
// nothing (they still take part in the cross-lane reduction).
// MU0 = 1 gives the Coulomb-gauge update: K from the spatial links only, G
// still applied to all 8 links; slice_active (optional, one flag per
// timeslice) leaves the sites of frozen timeslices untouched.
// OOP: the updated links go to out_field instead of back into field (every
// link has one end of each parity, so one half-sweep writes every link of
// out_field exactly once and the next half-sweep reads them from there).
// ACC: also g(x) <- G g(x) in the site field a.gacc (the accumulated gauge
// transformation of the mixed-precision bulk).
// MEAS: the written links are first reunitarized in FP64 and rounded to the
// storage format -- the values a separate reunitarization pass would store --
// and the site's F and theta contributions are taken from them: the forward
// links' Re tr into acc->f and tr[Delta Delta^dag] of x, from the new links
// around it (every one of them written by this update), into acc->th.
template <int F, int LPS, bool SR, bool NT, int MU0 = 0, bool OOP = false, bool ACC = false, bool MEAS = false>
__device__ __forceinline__ void update_site(void *__restrict__ field, const Geom &g, int parity, uint32_t h,
                                            int lane, bool active, const RelaxArgs<typename Fmt<F>::T> &a,
                                            const uint8_t *__restrict__ slice_active = nullptr,
                                            void *__restrict__ out_field = nullptr, MeasAcc *acc = nullptr)
{
    static_assert(!(OOP && MU0 != 0), "timeslice masks need the in-place update");
    static_assert(!(MEAS && MU0 != 0), "the fused measurement is the Landau one");
    using S = Fmt<F>;
    using T = typename S::T;
    constexpr int NL = 4 / LPS;  // directions handled per lane
    const Site c = decode(g, parity, h);
    if (slice_active) {
        // a frozen timeslice is neither read nor written; with one lane per
        // site no other lane waits on this one
        if (LPS == 1 && !slice_active[c.t]) return;
        active = active && slice_active[c.t];
    }

    mat3<T> uf[NL], ub[NL];
    uint32_t hb[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int mu = lane + k * LPS;
        hb[k] = back_half(g, c, h, mu);
        load_link<F, NT>(uf[k], block_ptr<F>(field, g.Vh, parity, mu), g.Vh, h);
        load_link<F, NT>(ub[k], block_ptr<F>(field, g.Vh, parity ^ 1, mu), g.Vh, hb[k]);
    }

    mat3<T> K;
    set_zero(K);
#pragma unroll
    for (int k = 0; k < NL; ++k)
        if (lane + k * LPS >= MU0) add_fwd_bwd(K, uf[k], ub[k]);
#pragma unroll
    for (int m = 1; m < LPS; m <<= 1)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                K.e[i][j].re += shfl_xor_t(K.e[i][j].re, m);
                K.e[i][j].im += shfl_xor_t(K.e[i][j].im, m);
            }

    bool sq0 = false, sq1 = false, sq2 = false;
    if constexpr (SR) {
        const uint32_t sweep = a.sweep_base ? (uint32_t)(*a.sweep_base + a.sweep) : a.sweep;
        const uint4 w = philox4x32_10(make_uint4(lex_index(g, c), sweep, a.instance, 3u), a.key0, a.key1);
        sq0 = (uint64_t)w.x < a.sr_threshold;
        sq1 = (uint64_t)w.y < a.sr_threshold;
        sq2 = (uint64_t)w.z < a.sr_threshold;
    }

    mat3<T> G;
    set_identity(G);
    const bool orl = a.overrelax != 0;
    su2_step<0, 1, true>(K, G, a.omega, orl, sq0);
    su2_step<0, 2, true>(K, G, a.omega, orl, sq1);
    su2_step<1, 2, false>(K, G, a.omega, orl, sq2);

    if (!active) return;
    if constexpr (ACC) {
        if (lane == 0) {
            // g(x) <- G g(x): the product of every update applied to this site
            mat3<T> gx, r;
            load_link<F>(gx, site_field_ptr<F>(a.gacc, g.Vh, parity), g.Vh, h);
            left_mul<S::R>(r, G, gx);
            store_link<F>(site_field_ptr<F>(a.gacc, g.Vh, parity), g.Vh, h, r);
        }
    }
    mat3<double> Kn;
    if constexpr (MEAS) set_zero(Kn);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int mu = lane + k * LPS;
        mat3<T> r, rb;
        left_mul<S::R>(r, G, uf[k]);
        right_mul_dag<S::R>(rb, ub[k], G);
        if constexpr (MEAS) {
            // only rows 0 and 1 enter the reunitarization, so the 12-real
            // products (rows 0 and 1) need no row 2 here
            mat3<double> df, db;
            convert(df, r);
            convert(db, rb);
            reunitarize(df);
            reunitarize(db);
            round_to_format<F>(df, r);
            round_to_format<F>(db, rb);
            acc->f += df.e[0][0].re + df.e[1][1].re + df.e[2][2].re;
            add_fwd_bwd(Kn, df, db);
        }
        store_link<F, NT>(block_ptr<F>(OOP ? out_field : field, g.Vh, parity, mu), g.Vh, h, r);
        store_link<F, NT>(block_ptr<F>(OOP ? out_field : field, g.Vh, parity ^ 1, mu), g.Vh, hb[k], rb);
    }
    if constexpr (MEAS) {
#pragma unroll
        for (int m = 1; m < LPS; m <<= 1)
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    Kn.e[i][j].re += shfl_xor_t(Kn.e[i][j].re, m);
                    Kn.e[i][j].im += shfl_xor_t(Kn.e[i][j].im, m);
                }
        if (lane == 0) acc->th += theta_of_K(Kn);
    }
}

// ----------------------------------------------------------------------------
// Fixed-link form of the sweep.  The links U keep their input values and the
// sweep updates the gauge transformation g instead; the link in the current
// gauge, g(x) U_mu(x) g(x+mu)^dag (Eq. (3)), exists only in registers.  With
// those links the K(x) of Eq. (8) factorises as
//   K(x) = g(x) M(x),  M(x) = sum_mu U_mu(x) g(x+mu)^dag + [g(x-mu) U_mu(x-mu)]^dag,
// so a site update reads its 8 links and the 8 neighbouring g of the other
// parity, runs the same three SU(2) steps on K starting from G = g(x), and
// stores only the new g(x).  A half-sweep moves 8 links in and one g in and
// out per site instead of 8 links in and out; the neighbouring g are shared by
// 8 sites each and mostly come from the caches.
// ----------------------------------------------------------------------------

// acc += p (all 9 entries)
template <typename T> __device__ __forceinline__ void add_to(mat3<T> &acc, const mat3<T> &p)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc.e[i][j] = acc.e[i][j] + p.e[i][j];
}

// acc += p^dag
template <typename T> __device__ __forceinline__ void add_dag_to(mat3<T> &acc, const mat3<T> &p)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc.e[i][j] = acc.e[i][j] + conj(p.e[j][i]);
}

// Re tr[a b]
__device__ __forceinline__ double re_tr_mul(const mat3<double> &a, const mat3<double> &b)
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) s += a.e[i][k].re * b.e[k][i].re - a.e[i][k].im * b.e[k][i].im;
    return s;
}

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The products of the fixed-link update as explicit multiply-add chains (the
// complex operators round every product and sum separately): rows [0, R) of
// r = u y^dag ...
template <int R, typename T>
__device__ __forceinline__ void mul_dag_fma(mat3<T> &r, const mat3<T> &u, const mat3<T> &y)
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T re = u.e[i][0].re * y.e[j][0].re, im = u.e[i][0].im * y.e[j][0].re;
            re = fmadd(u.e[i][0].im, y.e[j][0].im, re);
            im = fmadd(-u.e[i][0].re, y.e[j][0].im, im);
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                re = fmadd(u.e[i][k].re, y.e[j][k].re, re);
                re = fmadd(u.e[i][k].im, y.e[j][k].im, re);
                im = fmadd(u.e[i][k].im, y.e[j][k].re, im);
                im = fmadd(-u.e[i][k].re, y.e[j][k].im, im);
            }
            r.e[i][j] = {re, im};
        }
}

// ... rows [0, R) of r = y u ...
template <int R, typename T>
__device__ __forceinline__ void mul_fma(mat3<T> &r, const mat3<T> &y, const mat3<T> &u)
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T re = y.e[i][0].re * u.e[0][j].re, im = y.e[i][0].re * u.e[0][j].im;
            re = fmadd(-y.e[i][0].im, u.e[0][j].im, re);
            im = fmadd(y.e[i][0].im, u.e[0][j].re, im);
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                re = fmadd(y.e[i][k].re, u.e[k][j].re, re);
                re = fmadd(-y.e[i][k].im, u.e[k][j].im, re);
                im = fmadd(y.e[i][k].re, u.e[k][j].im, im);
                im = fmadd(y.e[i][k].im, u.e[k][j].re, im);
            }
            r.e[i][j] = {re, im};
        }
}

// ... and row 2 = conj(row0 x row1), the last row of an SU(3) matrix
template <typename T> __device__ __forceinline__ void row2_fma(mat3<T> &m)
{
    auto cross = [&](int a, int b, int c, int d) {  // conj(m0a m1b - m0c m1d)
        const cpx<T> A = m.e[0][a], B = m.e[1][b], C = m.e[0][c], D = m.e[1][d];
        T re = C.im * D.im;
        re = fmadd(-C.re, D.re, re);
        re = fmadd(-A.im, B.im, re);
        re = fmadd(A.re, B.re, re);
        T s = C.re * D.im;
        s = fmadd(C.im, D.re, s);
        T im = fmadd(A.re, B.im, -s);
        im = fmadd(A.im, B.re, im);
        return cpx<T>{re, -im};
    };
    m.e[2][0] = cross(1, 2, 2, 1);
    m.e[2][1] = cross(2, 0, 0, 2);
    m.e[2][2] = cross(0, 1, 1, 0);
}

// dst <- src on rows [0, R)
template <int R, typename A, typename B>
__device__ __forceinline__ void convert_rows(mat3<B> &dst, const mat3<A> &src)
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) dst.e[i][j] = {B(src.e[i][j].re), B(src.e[i][j].im)};
}

// The measurement's FP64 terms of M, from the operands exactly as the update
// holds them (u: rows [0, R); y: all rows): acc += u y^dag (forward) and
// acc += (y u)^dag (backward, y: rows [0, R); u: all rows).  In the FP64
// formats they are the update's own products bit for bit.
template <int R, typename T>
__device__ __forceinline__ void meas_term_fwd(mat3<double> &acc, const mat3<T> &u, const mat3<T> &y)
{
    mat3<double> ud, yd, pd;
    convert_rows<R>(ud, u);
    convert(yd, y);
    mul_dag_fma<R>(pd, ud, yd);
    if constexpr (R == 2) row2_fma(pd);
    add_to(acc, pd);
}

template <int R, typename T>
__device__ __forceinline__ void meas_term_bwd(mat3<double> &acc, const mat3<T> &y, const mat3<T> &u)
{
    mat3<double> yd, ud, pd;
    convert_rows<R>(yd, y);
    convert(ud, u);
    mul_fma<R>(pd, yd, ud);
    if constexpr (R == 2) row2_fma(pd);
    add_dag_to(acc, pd);
}

template <int LPS, typename T> __device__ __forceinline__ void lane_sum(mat3<T> &m)
{
#pragma unroll
    for (int s = 1; s < LPS; s <<= 1)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                m.e[i][j].re += shfl_xor_t(m.e[i][j].re, s);
                m.e[i][j].im += shfl_xor_t(m.e[i][j].im, s);
            }
}

// link mu of parity-`parity` site h for the fixed-link sweep in format F
// (kF64_12S: from the split storage; row 2 left unset)
template <int F>
__device__ __forceinline__ void load_fixed_link(mat3<typename Fmt<F>::T> &u, void *links, uint32_t Vh, int parity,
                                                int mu, uint32_t h)
{
    if constexpr (F == kF64_12S) load_link_split<true>(u, links, Vh, parity, mu, h);
    else load_link<F, true, false>(u, block_ptr<F>(links, Vh, parity, mu), Vh, h);
}

// The update of site h of the given parity in the fixed-link form, LPS lanes
// per site (each gathers the terms of 4 / LPS directions; M is summed over the
// lanes, every lane then runs the SU(2) steps and lane 0 stores).  links and
// the site field gf are in format F (kF64_12S: gf in FP64-12, the links in
// the split storage).
// POST = 1: the new g(x) is reunitarized in FP64 and rounded to the format
// before it is stored.  POST = 2: as 1, and the site's contributions to F and
// theta, from the links formed with the stored g(x) and the stored
// neighbours, go to acc (Re tr of its 4 forward links, tr[Delta Delta^dag]).
// MU0 = 1: the Coulomb-gauge update, M from the spatial directions only (the
// temporal links are not read at all); slice_active (optional, one flag per
// timeslice) leaves the sites of frozen timeslices alone -- the LPS lanes of
// a site share its timeslice, so they leave together.
// REC: links holds the per-site link records of format F (12-real or split; the
// same values, so the same arithmetic and bits as from the link field).
template <int F, int LPS, bool SR, int POST, int MU0 = 0, bool REC = false>
__device__ __forceinline__ void update_site_fixed(const void *__restrict__ links, void *__restrict__ gf,
                                                  const Geom &g, int parity, uint32_t h, int lane, bool active,
                                                  const RelaxArgs<typename Fmt<F>::T> &a, MeasAcc *acc,
                                                  const uint8_t *__restrict__ slice_active = nullptr)
{
    static_assert(!(POST == 2 && MU0 != 0), "the fused measurement is the Landau one");
    using S = Fmt<F>;
    using T = typename S::T;
    constexpr int NL = 4 / LPS;
    void *U = const_cast<void *>(links);
    const typename S::V *gn = site_field_ptr<F>(gf, g.Vh, parity ^ 1);
    const Site c = decode(g, parity, h);
    if (slice_active && !slice_active[c.t]) return;

    mat3<T> M;
    set_zero(M);
    mat3<double> Mf, Mb;  // POST == 2: forward (and in FP32 formats backward) terms in FP64
    if constexpr (POST == 2) {
        set_zero(Mf);
        set_zero(Mb);
    }
    // In the 12-real formats only rows 0 and 1 of each product are multiplied
    // out; row 2 of a product of two SU(3) matrices is conj(row0 x row1).
    constexpr int R = S::R;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int mu = lane + k * LPS;
        if (mu < MU0) continue;
        mat3<T> u, y, p;
        if constexpr (REC) load_link_rec<F>(u, U, g.Vh, parity, mu, h);
        else load_fixed_link<F>(u, U, g.Vh, parity, mu, h);
        load_link<F, false, false>(y, gn, g.Vh, fwd_half(g, c, h, mu));
        if constexpr (R == 2) row2_fma(y);
        mul_dag_fma<R>(p, u, y);  // U_mu(x) g(x+mu)^dag
        if constexpr (R == 2) row2_fma(p);
        add_to(M, p);
        if constexpr (POST == 2) {
            if constexpr (sizeof(T) == sizeof(double)) add_to(Mf, p);
            else meas_term_fwd<R>(Mf, u, y);
        }
        const uint32_t hb = back_half(g, c, h, mu);
        if constexpr (REC) load_link_rec<F>(u, U, g.Vh, parity, 4 + mu, h);
        else load_fixed_link<F>(u, U, g.Vh, parity ^ 1, mu, hb);
        load_link<F, false, false>(y, gn, g.Vh, hb);
        if constexpr (R == 2) row2_fma(u);
        mul_fma<R>(p, y, u);  // g(x-mu) U_mu(x-mu)
        if constexpr (R == 2) row2_fma(p);
        add_dag_to(M, p);
        // (FP64 formats: the backward terms are in M already; see below)
        if constexpr (POST == 2 && sizeof(T) != sizeof(double)) meas_term_bwd<R>(Mb, y, u);
    }
    lane_sum<LPS>(M);
    if constexpr (POST == 2) {
        lane_sum<LPS>(Mf);
        if constexpr (sizeof(T) != sizeof(double)) lane_sum<LPS>(Mb);
    }

    bool sq0 = false, sq1 = false, sq2 = false;
    if constexpr (SR) {
        const uint32_t sweep = a.sweep_base ? (uint32_t)(*a.sweep_base + a.sweep) : a.sweep;
        const uint4 w = philox4x32_10(make_uint4(lex_index(g, c), sweep, a.instance, 3u), a.key0, a.key1);
        sq0 = (uint64_t)w.x < a.sr_threshold;
        sq1 = (uint64_t)w.y < a.sr_threshold;
        sq2 = (uint64_t)w.z < a.sr_threshold;
    }

    typename S::V *gx = site_field_ptr<F>(gf, g.Vh, parity);
    mat3<T> G, K;
    load_link<F, true, false>(G, gx, g.Vh, h);
    if constexpr (R == 2) row2_fma(G);
    mul_fma<3>(K, G, M);
    const bool orl = a.overrelax != 0;
    su2_step<0, 1, true>(K, G, a.omega, orl, sq0);
    su2_step<0, 2, true>(K, G, a.omega, orl, sq1);
    su2_step<1, 2, false>(K, G, a.omega, orl, sq2);

    if constexpr (POST >= 1) {
        mat3<double> Gd;
        convert(Gd, G);
        reunitarize(Gd);
        round_to_format<F>(Gd, G);
        if constexpr (POST == 2) {
            // K of the stored g(x): in the FP64 formats from the update's own M
            // (its terms are the measurement's, summed in the update's order),
            // in the FP32 formats from the FP64 terms
            mat3<double> Md, Kn;
            if constexpr (sizeof(T) == sizeof(double)) {
                convert(Md, M);
            } else {
                Md = Mf;
                add_to(Md, Mb);
            }
            mul_fma<3>(Kn, Gd, Md);
            if (active && lane == 0) {
                acc->f += re_tr_mul(Gd, Mf);
                acc->th += theta_of_K(Kn);
            }
        }
    }
    if (active && lane == 0) store_link<F, true>(gx, g.Vh, h, G);
}

// Site h's F and theta contributions in the fixed-link form (read only, FP64),
// LPS lanes per site: f = sum_mu Re tr[g(x) U_mu(x) g(x+mu)^dag] and th =
// tr[Delta Delta^dag] of K(x) = g(x) M(x), every term of M formed as the
// update forms it (meas_term_fwd / _bwd) and g(x) with row 2 rebuilt as a
// store-and-load rebuilds it, so that the fused measurement of a sweep gets
// the same terms.  Only lane 0 of an active site returns non-zero sums.
// MU0 = 1: the Coulomb-gauge F_C and theta_C contributions (spatial links).
// REC: links holds the per-site link records (as in update_site_fixed).
template <int F, int LPS, int MU0 = 0, bool REC = false>
__device__ __forceinline__ void measure_site_fixed(const void *__restrict__ links, const void *__restrict__ gf,
                                                   const Geom &g, int parity, uint32_t h, int lane, bool active,
                                                   double &f, double &th)
{
    using S = Fmt<F>;
    using T = typename S::T;
    constexpr int R = S::R;
    void *U = const_cast<void *>(links);
    void *G = const_cast<void *>(gf);
    const typename S::V *gn = site_field_ptr<F>(G, g.Vh, parity ^ 1);
    const Site c = decode(g, parity, h);
    mat3<double> Mf, Mb;
    set_zero(Mf);
    set_zero(Mb);
#pragma unroll
    for (int k = 0; k < 4 / LPS; ++k) {
        const int mu = lane + k * LPS;
        if (mu < MU0) continue;
        mat3<T> u, y;
        if constexpr (REC) load_link_rec<F>(u, U, g.Vh, parity, mu, h);
        else load_fixed_link<F>(u, U, g.Vh, parity, mu, h);
        load_link<F, false, false>(y, gn, g.Vh, fwd_half(g, c, h, mu));
        if constexpr (R == 2) row2_fma(y);
        meas_term_fwd<R>(Mf, u, y);
        const uint32_t hb = back_half(g, c, h, mu);
        if constexpr (REC) load_link_rec<F>(u, U, g.Vh, parity, 4 + mu, h);
        else load_fixed_link<F>(u, U, g.Vh, parity ^ 1, mu, hb);
        load_link<F, false, false>(y, gn, g.Vh, hb);
        if constexpr (R == 2) row2_fma(u);
        meas_term_bwd<R>(Mb, y, u);
    }
    lane_sum<LPS>(Mf);
    lane_sum<LPS>(Mb);
    mat3<T> xt;
    load_link<F>(xt, site_field_ptr<F>(G, g.Vh, parity), g.Vh, h);
    mat3<double> x, Md = Mf, K;
    convert(x, xt);
    add_to(Md, Mb);
    mul_fma<3>(K, x, Md);
    const bool own = active && lane == 0;
    f = own ? re_tr_mul(x, Mf) : 0.0;
    th = own ? theta_of_K(K) : 0.0;
}

// ----------------------------------------------------------------------------
// F and theta (Eqs. (2), (4), (5)), optionally fused with reunitarization.
// Delta(x) = [(K - K^dag)/(2i)]_traceless, which equals sum_mu A_mu(x) -
// A_mu(x - mu) for A_mu = [(U - U^dag)/(2i)]_traceless.  All in FP64.
// ----------------------------------------------------------------------------

constexpr int kMeasureBlock = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// sums of a and b over a workgroup of any multiple of 64 lanes up to 256,
// in a fixed order, into out[0], out[1] (written by lane 0)
__device__ __forceinline__ void block_sum2_any(double a, double b, double *out)
{
    __shared__ double sa[4], sb[4];
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { sa[w] = a; sb[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) { ta += sa[i]; tb += sb[i]; }
        out[0] = ta;
        out[1] = tb;
    }
}

template <int BLOCK>
__device__ __forceinline__ void block_sum2(double a, double b, double *out)
{
    __shared__ double sa[BLOCK / 64], sb[BLOCK / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { sa[w] = a; sb[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
#pragma unroll
        for (int i = 0; i < BLOCK / 64; ++i) { ta += sa[i]; tb += sb[i]; }
        out[0] = ta;
        out[1] = tb;
    }
}

// Site h's contributions f = sum_mu Re tr U_mu(x) and th = |Delta(x)|^2.
// reunit_fwd: reunitarize the 4 forward links and store them; reunit_bwd:
// reunitarize the backward links in registers only (first parity pass,
// whose backward links are the other parity's not yet reunitarized forward
// links).  Inactive lanes return zeros and store nothing.  MU0 = 1 measures
// the Coulomb-gauge functional and precision (spatial links only), while the
// temporal forward links are still reunitarized when asked.
template <int F, int MU0 = 0>
__device__ __forceinline__ void measure_site(void *__restrict__ field, const Geom &g, int parity, uint32_t h,
                                             bool active, int reunit_fwd, int reunit_bwd, double &f, double &th)
{
    using S = Fmt<F>;
    using T = typename S::T;
    const Site c = decode(g, parity, h);
    f = 0.0;
    mat3<double> K;
    set_zero(K);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        mat3<T> ut, vt;
        load_link<F>(ut, block_ptr<F>(field, g.Vh, parity, mu), g.Vh, h);
        mat3<double> u, v;
        convert(u, ut);
        if (mu < MU0) {
            if (reunit_fwd) {
                reunitarize(u);
                mat3<T> o;
                round_to_format<F>(u, o);
                if (active) store_link<F>(block_ptr<F>(field, g.Vh, parity, mu), g.Vh, h, o);
            }
            continue;
        }
        load_link<F>(vt, block_ptr<F>(field, g.Vh, parity ^ 1, mu), g.Vh, back_half(g, c, h, mu));
        convert(v, vt);
        // Reunitarized links are measured exactly as they will be stored and
        // read back (rounded to the storage precision, row 2 rebuilt for the
        // 12-real formats), so the two parity passes agree bit for bit.
        if (reunit_fwd) {
            reunitarize(u);
            mat3<T> o;
            round_to_format<F>(u, o);
            if (active) store_link<F>(block_ptr<F>(field, g.Vh, parity, mu), g.Vh, h, o);
        }
        if (reunit_bwd) {
            reunitarize(v);
            mat3<T> o;
            round_to_format<F>(v, o);
        }
        f += u.e[0][0].re + u.e[1][1].re + u.e[2][2].re;
        add_fwd_bwd(K, u, v);
    }
    th = theta_of_K(K);
    if (!active) { f = 0.0; th = 0.0; }
}

}  // namespace lgf
