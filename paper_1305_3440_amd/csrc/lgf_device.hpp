// lgf_device.hpp -- device-side building blocks of the gfx950 gauge-fixing
// kernels: complex 3x3 algebra in registers, the storage formats and their
// parity-split structure-of-arrays layout, lattice geometry, Philox4x32-10.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lgf {

// ----------------------------------------------------------------------------
// Complex numbers and 3x3 complex matrices held in registers.
// ----------------------------------------------------------------------------

template <typename T> struct cpx { T re, im; };

template <typename T> __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
// a * conj(b)
template <typename T> __device__ __forceinline__ cpx<T> mul_conj(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T> __device__ __forceinline__ T norm2(cpx<T> a) { return a.re * a.re + a.im * a.im; }

template <typename T> struct mat3 { cpx<T> e[3][3]; };

template <typename T> __device__ __forceinline__ void set_identity(mat3<T> &a)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) a.e[i][j] = {T(i == j ? 1 : 0), T(0)};
}

template <typename T> __device__ __forceinline__ void set_zero(mat3<T> &a)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) a.e[i][j] = {T(0), T(0)};
}

// acc += u + v^dag
template <typename T>
__device__ __forceinline__ void add_fwd_bwd(mat3<T> &acc, const mat3<T> &u, const mat3<T> &v)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            acc.e[i][j].re += u.e[i][j].re + v.e[j][i].re;
            acc.e[i][j].im += u.e[i][j].im - v.e[j][i].im;
        }
}

// row 2 = conj(row0 x row1): the last row of a unitary matrix with det 1
template <typename T> __device__ __forceinline__ void rebuild_row2(mat3<T> &u)
{
    u.e[2][0] = conj(u.e[0][1] * u.e[1][2] - u.e[0][2] * u.e[1][1]);
    u.e[2][1] = conj(u.e[0][2] * u.e[1][0] - u.e[0][0] * u.e[1][2]);
    u.e[2][2] = conj(u.e[0][0] * u.e[1][1] - u.e[0][1] * u.e[1][0]);
}

// r = g * u, rows [0, R) only
template <int R, typename T>
__device__ __forceinline__ void left_mul(mat3<T> &r, const mat3<T> &g, const mat3<T> &u)
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.e[i][j] = g.e[i][0] * u.e[0][j] + g.e[i][1] * u.e[1][j] + g.e[i][2] * u.e[2][j];
}

// r = u * g^dag, rows [0, R) only
template <int R, typename T>
__device__ __forceinline__ void right_mul_dag(mat3<T> &r, const mat3<T> &u, const mat3<T> &g)
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.e[i][j] = mul_conj(u.e[i][0], g.e[j][0]) + mul_conj(u.e[i][1], g.e[j][1]) +
                        mul_conj(u.e[i][2], g.e[j][2]);
}

template <typename T> __device__ __forceinline__ T exact_rsqrt(T x);
// correctly rounded sqrt and division: the SU(2) normalisation amplifies
// rounding errors on ill-conditioned sites, so no approximate rsqrt here
template <> __device__ __forceinline__ float exact_rsqrt<float>(float x) { return 1.0f / sqrtf(x); }
template <> __device__ __forceinline__ double exact_rsqrt<double>(double x) { return 1.0 / sqrt(x); }

// Project a 3x3 matrix onto SU(3) in FP64: normalise row 0, orthogonalise
// and normalise row 1, row 2 = conj(row0 x row1).
__device__ __forceinline__ void reunitarize(mat3<double> &u)
{
    double n0 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) n0 += norm2(u.e[0][k]);
    const double i0 = 1.0 / sqrt(n0);
#pragma unroll
    for (int k = 0; k < 3; ++k) { u.e[0][k].re *= i0; u.e[0][k].im *= i0; }
    cpx<double> d = {0.0, 0.0};  // <row0, row1> = sum_k conj(row0_k) row1_k
#pragma unroll
    for (int k = 0; k < 3; ++k) d = d + conj(u.e[0][k]) * u.e[1][k];
#pragma unroll
    for (int k = 0; k < 3; ++k) u.e[1][k] = u.e[1][k] - d * u.e[0][k];
    double n1 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) n1 += norm2(u.e[1][k]);
    const double i1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int k = 0; k < 3; ++k) { u.e[1][k].re *= i1; u.e[1][k].im *= i1; }
    rebuild_row2(u);
}

template <typename A, typename B>
__device__ __forceinline__ void convert(mat3<B> &dst, const mat3<A> &src)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) dst.e[i][j] = {B(src.e[i][j].re), B(src.e[i][j].im)};
}

// ----------------------------------------------------------------------------
// Storage formats.  A field is split by parity; within a parity, direction
// and vector slot, the Vh = V/2 sites form one contiguous stream of 8- or
// 16-byte vectors ("planes"), so a wavefront's 64 consecutive sites load
// 512 B - 1 KB contiguous per instruction:
//     vector index = ((parity*4 + mu)*NV + slot)*Vh + h
// A link is stored row-major, (row, column, re/im), rows 0..R-1.
// ----------------------------------------------------------------------------

// kF64_12S: the fixed-link sweep in FP64 with g stored as FP64-12 and the
// read-only links in the split storage below (never a link field's format).
enum : int { kF64_18 = 0, kF32_18 = 1, kF32_12 = 2, kF64_12 = 3, kF64_12S = 4 };

typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <int F> struct Fmt;
template <> struct Fmt<kF64_18> { using T = double; using V = v2d; static constexpr int R = 3, NV = 9, CPV = 1; };
template <> struct Fmt<kF64_12> { using T = double; using V = v2d; static constexpr int R = 2, NV = 6, CPV = 1; };
template <> struct Fmt<kF32_18> { using T = float;  using V = v2f; static constexpr int R = 3, NV = 9, CPV = 1; };
template <> struct Fmt<kF32_12> { using T = float;  using V = v4f; static constexpr int R = 2, NV = 3, CPV = 2; };
template <> struct Fmt<kF64_12S> : Fmt<kF64_12> {};  // the site field g

// vector load / store, optionally marked non-temporal (streamed past the
// caches: every link is read and written once per half-sweep)
template <bool NT, typename V> __device__ __forceinline__ V vload(const V *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename V> __device__ __forceinline__ void vstore(V *p, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// base pointer of the (parity, mu) block
template <int F>
__device__ __forceinline__ typename Fmt<F>::V *block_ptr(void *field, uint32_t Vh, int parity, int mu)
{
    return reinterpret_cast<typename Fmt<F>::V *>(field) +
           (size_t)((parity * 4 + mu) * Fmt<F>::NV) * Vh;
}

// the NV vectors of one link, row-major, into a matrix (rows 0..R-1)
template <int F>
__device__ __forceinline__ void unpack_link(mat3<typename Fmt<F>::T> &u, const typename Fmt<F>::V *v)
{
    using S = Fmt<F>;
    if constexpr (S::CPV == 1) {
#pragma unroll
        for (int k = 0; k < S::NV; ++k) u.e[k / 3][k % 3] = {v[k].x, v[k].y};
    } else {
#pragma unroll
        for (int k = 0; k < S::NV; ++k) {
            u.e[(2 * k) / 3][(2 * k) % 3] = {v[k].x, v[k].y};
            u.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v[k].z, v[k].w};
        }
    }
}

// ROW2 = false leaves row 2 of a 12-real link unset (for callers that only
// read rows 0 and 1)
template <int F, bool NT = false, bool ROW2 = true>
__device__ __forceinline__ void load_link(mat3<typename Fmt<F>::T> &u, const typename Fmt<F>::V *blk,
                                          uint32_t Vh, uint32_t h)
{
    using S = Fmt<F>;
    typename S::V v[S::NV];
#pragma unroll
    for (int k = 0; k < S::NV; ++k) v[k] = vload<NT>(blk + (size_t)k * Vh + h);
    unpack_link<F>(u, v);
    if constexpr (S::R == 2 && ROW2) rebuild_row2(u);
}

// Split FP64 storage of read-only links: rows 0 and 1 of each link rounded
// to FP32, laid out as the FP32-12 field, followed by a second field of the
// same shape holding each element's remainder x - hi as a 16-bit integer q in
// units of 2^-40 (three 4 x int16 vectors per link).  The element read back,
// hi + q 2^-40, is exact in FP64 and within 2^-40 of x for |x| <= 1 (every
// entry of an SU(3) matrix): 72 B per link instead of 96 B in FP64-12.
typedef short v4s __attribute__((ext_vector_type(4)));
constexpr double kSplitUnit = 0x1p-40;

__device__ __forceinline__ v4s *split_res_ptr(void *field, uint32_t Vh, int parity, int mu)
{
    return reinterpret_cast<v4s *>(reinterpret_cast<v4f *>(field) + (size_t)24 * Vh) +
           (size_t)((parity * 4 + mu) * 3) * Vh;
}

__device__ __forceinline__ void split_encode(double x, float &hi, short &q)
{
    hi = (float)x;  // round to nearest, ties to even
    const double r = rint((x - (double)hi) * 0x1p40);  // x - hi is exact
    q = (short)fmin(fmax(r, -32767.0), 32767.0);
}

template <bool NT>
__device__ __forceinline__ void load_link_split(mat3<double> &u, void *field, uint32_t Vh, int parity, int mu,
                                                uint32_t h)
{
    const v4f *hb = block_ptr<kF32_12>(field, Vh, parity, mu);
    const v4s *qb = split_res_ptr(field, Vh, parity, mu);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const v4f a = vload<NT>(hb + (size_t)k * Vh + h);
        const v4s q = vload<NT>(qb + (size_t)k * Vh + h);
        u.e[(2 * k) / 3][(2 * k) % 3] = {(double)a.x + (double)q.x * kSplitUnit,
                                         (double)a.y + (double)q.y * kSplitUnit};
        u.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = {(double)a.z + (double)q.z * kSplitUnit,
                                                 (double)a.w + (double)q.w * kSplitUnit};
    }
}

// Per-site link records: a read-only copy of a 12-real link field for the
// sweeps that keep the links fixed.  For each parity, the sites are grouped
// in tiles of kRecTile consecutive half indices; a tile holds, for each of
// its sites, the 8 links one site update reads -- U_mu(x) in slot mu and
// U_mu(x - mu) in slot 4 + mu -- vector by vector across the tile's sites:
//     vector index = ((parity * rec_tiles(Vh) + h / T) * 8 + slot) * NV * T
//                    + k * T + h % T,    T = kRecTile, k < NV
// so the 8 links of a wavefront's 32 sites are one contiguous block (every
// link is stored twice, once with each end; a last partial tile is padded).
// kF64_12S records hold the split storage: per (parity, tile, slot) the 3
// FP32 vectors of the tile's links as above (NV = 3), then their 3 remainder
// vectors (v4s) in the same order, 72 B per link.
constexpr uint32_t kRecTile = 32;
__host__ __device__ inline uint32_t rec_tiles(uint32_t Vh) { return (Vh + kRecTile - 1) / kRecTile; }

// first FP32 vector and first remainder vector of link `slot` of site h in
// kF64_12S records
__device__ __forceinline__ const v4f *rec_split_hi(const void *rec, uint32_t Vh, int parity, int slot, uint32_t h)
{
    const size_t blk = ((size_t)parity * rec_tiles(Vh) + h / kRecTile) * 8 + (size_t)slot;
    return reinterpret_cast<const v4f *>(reinterpret_cast<const char *>(rec) + blk * (kRecTile * 72)) +
           h % kRecTile;
}
__device__ __forceinline__ const v4s *rec_split_lo(const void *rec, uint32_t Vh, int parity, int slot, uint32_t h)
{
    const size_t blk = ((size_t)parity * rec_tiles(Vh) + h / kRecTile) * 8 + (size_t)slot;
    return reinterpret_cast<const v4s *>(reinterpret_cast<const char *>(rec) + blk * (kRecTile * 72) +
                                         kRecTile * 48) +
           h % kRecTile;
}

template <int F>
__device__ __forceinline__ const typename Fmt<F>::V *rec_ptr(const void *rec, uint32_t Vh, int parity, int slot,
                                                             uint32_t h)
{
    return reinterpret_cast<const typename Fmt<F>::V *>(rec) +
           (((size_t)parity * rec_tiles(Vh) + h / kRecTile) * 8 + (size_t)slot) * Fmt<F>::NV * kRecTile +
           h % kRecTile;
}

// link `slot` of site h's record, rows 0 and 1 (streamed past the caches)
template <int F>
__device__ __forceinline__ void load_link_rec(mat3<typename Fmt<F>::T> &u, const void *rec, uint32_t Vh, int parity,
                                              int slot, uint32_t h)
{
    static_assert(Fmt<F>::R == 2, "records hold 12-real links");
    if constexpr (F == kF64_12S) {
        const v4f *hb = rec_split_hi(rec, Vh, parity, slot, h);
        const v4s *qb = rec_split_lo(rec, Vh, parity, slot, h);
        v4f a[3];
        v4s q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            a[k] = vload<true>(hb + (size_t)k * kRecTile);
            q[k] = vload<true>(qb + (size_t)k * kRecTile);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            u.e[(2 * k) / 3][(2 * k) % 3] = {(double)a[k].x + (double)q[k].x * kSplitUnit,
                                             (double)a[k].y + (double)q[k].y * kSplitUnit};
            u.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = {(double)a[k].z + (double)q[k].z * kSplitUnit,
                                                     (double)a[k].w + (double)q[k].w * kSplitUnit};
        }
    } else {
        const typename Fmt<F>::V *b = rec_ptr<F>(rec, Vh, parity, slot, h);
        typename Fmt<F>::V v[Fmt<F>::NV];
#pragma unroll
        for (int k = 0; k < Fmt<F>::NV; ++k) v[k] = vload<true>(b + (size_t)k * kRecTile);
        unpack_link<F>(u, v);
    }
}

template <int F, bool NT = false>
__device__ __forceinline__ void store_link(typename Fmt<F>::V *blk, uint32_t Vh, uint32_t h,
                                           const mat3<typename Fmt<F>::T> &u)
{
    using S = Fmt<F>;
#pragma unroll
    for (int k = 0; k < S::NV; ++k) {
        typename S::V v;
        if constexpr (S::CPV == 1) {
            v.x = u.e[k / 3][k % 3].re;
            v.y = u.e[k / 3][k % 3].im;
        } else {
            v.x = u.e[(2 * k) / 3][(2 * k) % 3].re;
            v.y = u.e[(2 * k) / 3][(2 * k) % 3].im;
            v.z = u.e[(2 * k + 1) / 3][(2 * k + 1) % 3].re;
            v.w = u.e[(2 * k + 1) / 3][(2 * k + 1) % 3].im;
        }
        vstore<NT>(blk + (size_t)k * Vh + h, v);
    }
}

// ----------------------------------------------------------------------------
// Lattice geometry.  Half index h of a site of parity p is floor(s/2) with
// s the lexicographic index (Lx even, so each x-row holds Lx/2 sites of each
// parity); the parity-(1-p) neighbours of x in the t, z, y directions sit at
// h -/+ the half strides, the x neighbours at the same row position or one off.
// ----------------------------------------------------------------------------

struct Geom {
    uint32_t L[4];   // Lt, Lz, Ly, Lx
    uint32_t hx;     // Lx / 2
    uint32_t Vh;     // V / 2
    uint32_t hs[3];  // half strides of t, z, y: Lz*Ly*hx, Ly*hx, hx
};

struct Site {
    uint32_t t, z, y, x;
    uint32_t row;  // (t*Lz + z)*Ly + y
};

__device__ __forceinline__ Site decode(const Geom &g, int parity, uint32_t h)
{
    Site c;
    c.row = h / g.hx;
    const uint32_t xh = h - c.row * g.hx;
    uint32_t r = c.row;
    c.y = r % g.L[2];
    r /= g.L[2];
    c.z = r % g.L[1];
    c.t = r / g.L[1];
    c.x = 2 * xh + ((parity + c.t + c.z + c.y) & 1u);
    return c;
}

// half index (in the other parity) of the site x - mu
__device__ __forceinline__ uint32_t back_half(const Geom &g, const Site &c, uint32_t h, int mu)
{
    if (mu == 3) {
        const uint32_t xb = (c.x == 0) ? g.L[3] - 1 : c.x - 1;
        return c.row * g.hx + (xb >> 1);
    }
    const uint32_t coord = (mu == 0) ? c.t : (mu == 1) ? c.z : c.y;
    const uint32_t ext = g.L[mu];
    const uint32_t hs = g.hs[mu];
    return (coord == 0) ? h + (ext - 1) * hs : h - hs;
}

// half index (in the other parity) of the site x + mu
__device__ __forceinline__ uint32_t fwd_half(const Geom &g, const Site &c, uint32_t h, int mu)
{
    if (mu == 3) {
        const uint32_t xf = (c.x + 1 == g.L[3]) ? 0 : c.x + 1;
        return c.row * g.hx + (xf >> 1);
    }
    const uint32_t coord = (mu == 0) ? c.t : (mu == 1) ? c.z : c.y;
    return (coord + 1 == g.L[mu]) ? h - (g.L[mu] - 1) * g.hs[mu] : h + g.hs[mu];
}

__device__ __forceinline__ uint32_t lex_index(const Geom &g, const Site &c) { return c.row * g.L[3] + c.x; }

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// (x0, x1, x2, x3) -> (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1,
// lo(M0 x0)) with the key bumped by the Weyl increments between rounds.
// ----------------------------------------------------------------------------

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = M0 * c.x, hi0 = __umulhi(M0, c.x);
        const uint32_t lo1 = M1 * c.z, hi1 = __umulhi(M1, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += W0;
        k1 += W1;
    }
    return c;
}

}  // namespace lgf
