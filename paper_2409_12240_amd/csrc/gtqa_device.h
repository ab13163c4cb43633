// Device helpers shared by the GTQA kernel sources: complex arithmetic in
// registers, cross-lane exchanges, butterfly reductions, the team Jacobi
// SVD and the incoming-message / lambda lookups of a site tensor.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gtqa_internal.h"

namespace gtqa {

// true when a tail_gate says that BP has not stopped (uniform per launch)
__device__ __forceinline__ bool tail_gated_off(const DevPool& p) {
    return p.tail_gate != nullptr && (p.tail_gate[0] | p.tail_gate[1]) != 0;
}

// ------------------------------------------------------------------ complex
template <typename R>
struct cpx {
    R re, im;
};
using cd = cpx<double>;

template <typename R>
__device__ __forceinline__ cpx<R> cz() { return {R(0), R(0)}; }
template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// conj(a) * b
template <typename R>
__device__ __forceinline__ cpx<R> ccmul(cpx<R> a, cpx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.re * s, a.im * s}; }
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ R cabs2(cpx<R> a) { return a.re * a.re + a.im * a.im; }
// acc + a*b
template <typename R>
__device__ __forceinline__ cpx<R> cfma(cpx<R> acc, cpx<R> a, cpx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
    return acc;
}
// acc + a*conj(b)
template <typename R>
__device__ __forceinline__ cpx<R> cfmac(cpx<R> acc, cpx<R> a, cpx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.im, b.re, acc.im);
    acc.im = fma(-a.re, b.im, acc.im);
    return acc;
}
// acc + conj(a)*b
template <typename R>
__device__ __forceinline__ cpx<R> ccfma(cpx<R> acc, cpx<R> a, cpx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
    return acc;
}

template <typename S>
__device__ __forceinline__ cd to_cd(cpx<S> x) { return {double(x.re), double(x.im)}; }
template <typename S>
__device__ __forceinline__ cpx<S> from_cd(cd x) { return {S(x.re), S(x.im)}; }

// ------------------------------------------------------------------ shuffles
// Xor lane exchanges built from VALU lane permutes (verified lane maps):
//   xor 1, 2, 3: DPP quad_perm; xor 7: DPP row_half_mirror; xor 15: DPP
//   row_mirror; xor 8: DPP row_ror:8; xor 16 / 32: v_permlane16_swap /
//   v_permlane32_swap.  All lanes of the segment the mask spans must be active.
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ int dpp_x1(int x) { return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_x2(int x) { return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_x8(int x) { return __builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false); }
__device__ __forceinline__ int perm_x16(int x) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return ((lane_id() >> 4) & 1) ? r[0] : r[1];
}
__device__ __forceinline__ int perm_x32(int x) {
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (lane_id() >> 5) ? r[0] : r[1];
}
__device__ __forceinline__ int dpp_x3(int x) { return __builtin_amdgcn_mov_dpp(x, 0x1B, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_x7(int x) { return __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_x15(int x) { return __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false); }
// Lane xor by a compile-time mask (wherever this is inlined in an unrolled
// loop).  Xor maps compose, so the low four bits take at most two DPP moves:
// quad reverse is xor 3, row half-mirror xor 7, row mirror xor 15, and
// row_ror:8 xor 8 within each 16-lane row.
__device__ __forceinline__ int xshfl_i(int x, int mask) {
    switch (mask & 15) {
        case 0: break;
        case 1: x = dpp_x1(x); break;
        case 2: x = dpp_x2(x); break;
        case 3: x = dpp_x3(x); break;
        case 4: x = dpp_x3(dpp_x7(x)); break;
        case 5: x = dpp_x2(dpp_x7(x)); break;
        case 6: x = dpp_x1(dpp_x7(x)); break;
        case 7: x = dpp_x7(x); break;
        case 8: x = dpp_x8(x); break;
        case 9: x = dpp_x1(dpp_x8(x)); break;
        case 10: x = dpp_x2(dpp_x8(x)); break;
        case 11: x = dpp_x3(dpp_x8(x)); break;
        case 12: x = dpp_x3(dpp_x15(x)); break;
        case 13: x = dpp_x2(dpp_x15(x)); break;
        case 14: x = dpp_x1(dpp_x15(x)); break;
        default: x = dpp_x15(x); break;
    }
    if (mask & 16) x = perm_x16(x);
    if (mask & 32) x = perm_x32(x);
    return x;
}
__device__ __forceinline__ double xshfl(double v, int mask) {
    const int lo = xshfl_i(__double2loint(v), mask);
    const int hi = xshfl_i(__double2hiint(v), mask);
    return __hiloint2double(hi, lo);
}

// Butterfly reductions over aligned W-lane segments, offsets W/2, W/4, ..., 1
// (written recursively so every shuffle mask is a literal constant).
template <int W>
__device__ __forceinline__ double seg_sum(double x) {
    if constexpr (W > 1) return seg_sum<W / 2>(x + xshfl(x, W / 2));
    else return x;
}
template <int W>
__device__ __forceinline__ cd seg_sum(cd x) {
    if constexpr (W > 1) return seg_sum<W / 2>(cd{x.re + xshfl(x.re, W / 2), x.im + xshfl(x.im, W / 2)});
    else return x;
}
template <int W>
__device__ __forceinline__ float seg_sum(float x) {
    if constexpr (W > 1) return seg_sum<W / 2>(x + __int_as_float(xshfl_i(__float_as_int(x), W / 2)));
    else return x;
}
template <int W>
__device__ __forceinline__ cpx<float> seg_sum(cpx<float> x) {
    return {seg_sum<W>(x.re), seg_sum<W>(x.im)};
}
// complex value of lane ^ mask (mask a constant after unrolling)
__device__ __forceinline__ cpx<float> wxor(cpx<float> v, int mask) {
    return {__int_as_float(xshfl_i(__float_as_int(v.re), mask)), __int_as_float(xshfl_i(__float_as_int(v.im), mask))};
}
__device__ __forceinline__ cd wxor(cd v, int mask) { return {xshfl(v.re, mask), xshfl(v.im, mask)}; }
template <int W>
__device__ __forceinline__ int seg_max(int x) {
    if constexpr (W > 1) return seg_max<W / 2>(max(x, xshfl_i(x, W / 2)));
    else return x;
}
// broadcast of lane s (0..3) of each aligned quad by DPP quad_perm; s must be
// a constant after unrolling
__device__ __forceinline__ int quad_bcast_i(int x, int s) {
    switch (s) {
        case 0: return __builtin_amdgcn_mov_dpp(x, 0x00, 0xF, 0xF, false);
        case 1: return __builtin_amdgcn_mov_dpp(x, 0x55, 0xF, 0xF, false);
        case 2: return __builtin_amdgcn_mov_dpp(x, 0xAA, 0xF, 0xF, false);
        default: return __builtin_amdgcn_mov_dpp(x, 0xFF, 0xF, 0xF, false);
    }
}
__device__ __forceinline__ double quad_bcast(double v, int s) {
    const int lo = quad_bcast_i(__double2loint(v), s);
    const int hi = quad_bcast_i(__double2hiint(v), s);
    return __hiloint2double(hi, lo);
}

// general lane gather (any source lane within a W-lane segment)
template <int W>
__device__ __forceinline__ cd shfl_cd(cd x, int src) {
    return {__shfl(x.re, src, W), __shfl(x.im, src, W)};
}

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// stride of leg l (0..2) in a [2][chi][chi][chi] site tensor
template <int CHI>
__device__ __forceinline__ int leg_stride(int l) { return l == 0 ? CHI * CHI : (l == 1 ? CHI : 1); }

// Work-group index in item order.  The dispatcher hands work-groups to the
// 8 XCDs round-robin; with p.xcd_remap the launch grid is a multiple of 8 and
// XCD x takes the contiguous item range [x G/8, (x+1) G/8), so the items of
// one instance (which share lambdas, messages and gauge maps) meet in one L2.
__device__ __forceinline__ int wg_index(int remap) {
    if (!remap) return (int)blockIdx.x;
    const int per = (int)gridDim.x >> 3;
    return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

// the two legs other than p, ascending
__device__ __forceinline__ void other_legs(int p, int& o1, int& o2) {
    o1 = (p == 0) ? 1 : 0;
    o2 = (p == 2) ? 1 : 2;
}

// ------------------------------------------------------------------ Jacobi SVD
// One-sided (Hestenes) Jacobi SVD of an N x N complex matrix (N a power of
// two) held by a team of TEAM lanes: lane t owns column c = t % N and rows
// g + LPC*k (g = t / N, k < EPL).  Round r = 1..N-1 of a sweep pairs
// column c with column c ^ r, which sits in lane t ^ r: every pair meets
// once per sweep and the partner's data is one xor-shuffle away, with masks
// below 16 (at most two DPP moves each); a column's LPC lanes are t ^ (N j).  Column norms are recomputed at
// the start of each sweep and carried through the rotations
// (alpha' = alpha - t|gamma|, beta' = beta + t|gamma|).  On return the
// columns of m are A V (orthogonal; their norms are the singular values) and
// v holds V (if WANT_V).  Returns the sweeps used, max_sweeps + 1 if the cap
// was hit.
template <int N, int TEAM>
struct JLayout {
    static constexpr int LPC = TEAM / N;
    static constexpr int EPL = N / LPC;
    static_assert((N & (N - 1)) == 0, "N must be a power of two");
    static_assert(LPC >= 1 && LPC * N == TEAM, "team must be a multiple of N");
    static_assert(EPL * LPC == N, "rows must divide evenly");
    __device__ static int col(int t) { return t % N; }
    __device__ static int grp(int t) { return t / N; }
};

// Sum over the CNT lanes t ^ (STRIDE j), j < CNT (CNT a power of two): the
// lanes of one Jacobi column when STRIDE = N.
template <int STRIDE, int CNT>
__device__ __forceinline__ double strided_sum(double x) {
    if constexpr (CNT > 1) return strided_sum<STRIDE, CNT / 2>(x + xshfl(x, STRIDE * (CNT / 2)));
    else return x;
}
template <int STRIDE, int CNT>
__device__ __forceinline__ cd strided_sum(cd x) {
    if constexpr (CNT > 1)
        return strided_sum<STRIDE, CNT / 2>(cd{x.re + xshfl(x.re, STRIDE * (CNT / 2)),
                                               x.im + xshfl(x.im, STRIDE * (CNT / 2))});
    else return x;
}

__device__ __forceinline__ cd shfl_xor_cd(cd x, int mask) {
    return {xshfl(x.re, mask), xshfl(x.im, mask)};
}

// The value of lane addr / 4 through the LDS crossbar (ds_bpermute): one
// instruction per dword, none on the VALU, for any lane map.
__device__ __forceinline__ double bperm_d(double v, int addr) {
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cd bperm_cd(cd x, int addr) { return {bperm_d(x.re, addr), bperm_d(x.im, addr)}; }

// Rank of this lane's column among the N columns by squared norm `own`
// (descending, ties by column index); every lane of a column gets the same.
template <int N, int LPC>
__device__ __forceinline__ int column_rank(double own, int col) {
    int rank = 0;
#pragma unroll
    for (int r = 1; r < N; ++r) {
        const double o = xshfl(own, r);
        rank += (o > own || (o == own && (col ^ r) < col)) ? 1 : 0;
    }
    return rank;
}

// With KEEP < N only pairs that involve one of the KEEP largest columns (by
// norm at the start of the sweep) are rotated.  At convergence those columns
// are orthogonal to every other column, so they are exact singular vectors
// times singular values, while the other columns span the complement: their
// total squared norm is exact, their individual norms are not singular
// values.  Callers that keep only the leading KEEP triplets (truncation)
// skip the sweeps that would orthogonalise the discarded ones among
// themselves; kept_set_is_largest below checks that the kept values are the
// KEEP largest, and the caller redoes the decomposition on every pair when
// they are not.
constexpr int KEEP_SWEEPS = 16;

template <int W>
__device__ __forceinline__ double seg_min(double x) {
    if constexpr (W > 1) return seg_min<W / 2>(fmin(x, xshfl(x, W / 2)));
    else return x;
}
template <int W>
__device__ __forceinline__ double seg_maxd(double x) {
    if constexpr (W > 1) return seg_maxd<W / 2>(fmax(x, xshfl(x, W / 2)));
    else return x;
}

// REFETCH: the partner column is fetched twice per round (for gamma and
// again for the rotation) instead of being held, which halves the registers
// the round needs at twice its cross-lane moves (used where occupancy, not
// issue, limits the team); the fetches go through LDS lane permutes, which
// take no VALU issue slots, where the DPP / permlane forms of most masks
// take two to four VALU instructions and hazard waits per dword.
template <int N, int TEAM, bool WANT_V = true, int KEEP = N, bool REFETCH = false>
__device__ __forceinline__ int jacobi_svd_team(cd* m, cd* v, int t, double tol, int max_sweeps) {
    constexpr int LPC = JLayout<N, TEAM>::LPC;
    constexpr int EPL = JLayout<N, TEAM>::EPL;
    const int col = JLayout<N, TEAM>::col(t);
    const double tol2 = tol * tol;
    // A sweep whose rotations all have |gamma| <= eps sqrt(alpha beta) and
    // sine <= eps leaves every pair with relative |gamma| below about
    // 2 (N - 2) eps^2 (each later rotation moves a pair's gamma by at most a
    // sine times another relative gamma); with eps^2 = tol / (20 (N - 2))
    // that is under tol / 10, so the sweep that would only confirm
    // convergence is skipped.
    const double eps2 = tol / (20.0 * (N - 2 > 0 ? N - 2 : 1));
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double own = 0.0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) own += cabs2(m[k]);
        own = strided_sum<N, LPC>(own);
        const bool kept = KEEP >= N || column_rank<N, LPC>(own, col) < KEEP;
        int rotated = 0, big = 0;
#pragma unroll
        for (int r = 1; r < N; ++r) {
            const int mask = r;
            cd pm[REFETCH ? 1 : EPL], pv[EPL];
            if constexpr (!REFETCH) {
#pragma unroll
                for (int k = 0; k < EPL; ++k) {
                    pm[k] = shfl_xor_cd(m[k], mask);
                    if (WANT_V) pv[k] = shfl_xor_cd(v[k], mask);
                }
            }
            const double par = xshfl(own, mask);
            const int paddr = (lane_id() ^ mask) << 2;          // REFETCH: partner lane, in bytes
            // the pair (p, q), p < q: this lane holds column p iff its column
            // lacks the highest bit of r
            const bool is_p = (col ^ r) > col;
            // gl = conj(own column) . partner: gamma = m_p^H m_q on the p side,
            // conj(gamma) on the q side.  The imaginary part is the difference
            // of two separately accumulated sums, which trade places between
            // the two sides, so the q side holds exactly conj of the p side
            // (a single fused chain would round the two sides differently, and
            // the two halves of the rotation would then not match).
            cd gl;
            {
                double re = 0.0, pa = 0.0, pb = 0.0;
#pragma unroll
                for (int k = 0; k < EPL; ++k) {
                    const cd q = REFETCH ? bperm_cd(m[k], paddr) : pm[REFETCH ? 0 : k];
                    re = fma(m[k].re, q.re, re);
                    re = fma(m[k].im, q.im, re);
                    pa = fma(m[k].re, q.im, pa);
                    pb = fma(m[k].im, q.re, pb);
                }
                gl = {re, pa - pb};
            }
            gl = strided_sum<N, LPC>(gl);
            // sg = +1 on the p side, -1 on the q side; every pair quantity
            // below comes out bitwise equal in both lanes of the pair
            const double sg = is_p ? 1.0 : -1.0;
            const double g2 = cabs2(gl);
            const bool pkept = KEEP >= N || xshfl_i(kept ? 1 : 0, mask) != 0;
            const bool rot = g2 > 0.0 && g2 > tol2 * (own * par) && (kept || pkept);
            rotated |= rot ? 1 : 0;
            // [m_p, m_q] <- [c m_p - conj(S) m_q, S m_p + c m_q] with S = c tau gamma
            // and c = (1 + tau^2 |gamma|^2)^(-1/2): unitary for any real tau.
            // tau = sign(d) / (|d| + sqrt(d^2 + |gamma|^2)), d = (|m_q|^2 - |m_p|^2)/2,
            // zeroes m_p^H m_q; hardware approximations suffice for it.
            // (d is -0 in the q lane where the p lane has +0: the sign is
            // taken by comparison, so both lanes agree)
            const double d = (0.5 * sg) * (par - own);
            const double x = fma(d, d, g2);
            const double den = fabs(d) + x * __builtin_amdgcn_rsq(x);
            const double rden = __builtin_amdgcn_rcp(den);
            const double tau = rot ? (d >= 0.0 ? rden : -rden) : 0.0;
            const double tg = tau * g2;
            const double ts = tau * tg;                        // tan^2 of the angle
            // c = (1 + ts)^(-1/2) to full precision: the hardware estimate
            // (relative error ~5e-8) and one Newton step with its second-order
            // term, y (1 + e/2 + 3e^2/8), e = 1 - a y^2 (measured within
            // 1.4e-16 of the exact value, as the library routine); a >= 1 is
            // finite, so no special values arise
            const double a1 = 1.0 + ts;
            const double y0 = __builtin_amdgcn_rsq(a1);
            const double er = fma(-a1 * y0, y0, 1.0);
            const double c = fma(y0 * er, fma(er, 0.375, 0.5), y0);
            const double bs = -(sg * c) * tau;                 // B = bs * conj(gl)
            big |= (rot && (g2 > eps2 * (own * par) || ts > eps2)) ? 2 : 0;
            const cd B = {bs * gl.re, -bs * gl.im};
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                if constexpr (REFETCH) {
                    const cd q = bperm_cd(m[k], paddr);
                    m[k] = cfma(cscale(m[k], c), B, q);
                    if (WANT_V) {
                        const cd qv = bperm_cd(v[k], paddr);
                        v[k] = cfma(cscale(v[k], c), B, qv);
                    }
                } else {
                    m[k] = cfma(cscale(m[k], c), B, pm[k]);
                    if (WANT_V) v[k] = cfma(cscale(v[k], c), B, pv[k]);
                }
            }
            own = fma(-sg, tg, own);
        }
        // 0: nothing rotated; 1: only rotations below the quadratic bound,
        // which ends the iteration only if the kept set is still the same
        int st = seg_max<TEAM>(rotated | big);
        if (KEEP < N && st == 1) {
            const bool kept_now = column_rank<N, LPC>(own, col) < KEEP;
            st = seg_max<TEAM>(kept_now != kept ? 2 : 1);
        }
        if (st < 2) return sweep + 1;
    }
    return max_sweeps + 1;
}

// After a KEEP < N run: are the KEEP largest columns the KEEP largest
// singular values?  The discarded columns are orthogonal to the kept ones, so
// their largest singular value is at most their Frobenius norm; the answer
// is yes when their total squared norm lies below the smallest kept squared
// norm, or below (cut_rel sigma_max)^2 (every discarded value is dropped by
// the relative cutoff anyway).  Uniform over the team: every value is
// reduced by butterflies, which leave bitwise equal results in all lanes.
template <int N, int TEAM, int KEEP>
__device__ bool kept_set_is_largest(const cd* m, int t, double cut_rel) {
    constexpr int LPC = JLayout<N, TEAM>::LPC;
    constexpr int EPL = JLayout<N, TEAM>::EPL;
    const int col = JLayout<N, TEAM>::col(t);
    double o = 0.0;
#pragma unroll
    for (int k = 0; k < EPL; ++k) o += cabs2(m[k]);
    o = strided_sum<N, LPC>(o);
    const bool kp = column_rank<N, LPC>(o, col) < KEEP;
    // the N lanes t ^ r (r < N) hold the N columns once each
    const double dsum = seg_sum<N>(kp ? 0.0 : o);
    const double kmin = seg_min<N>(kp ? o : __builtin_huge_val());
    const double omax = seg_maxd<N>(o);
    return dsum < kmin || dsum <= (cut_rel * cut_rel) * omax;
}

constexpr double JACOBI_TOL = 1e-15;
constexpr int JACOBI_MAX_SWEEPS = 40;

// incoming message at vertex a along its leg l: pointer + whether virtual
template <typename S>
__device__ __forceinline__ const cpx<S>* incoming_msg(const DevPool& p, int a, int l, int CHI) {
    const int e2 = p.vedge[3 * a + l];
    if (e2 < 0) return nullptr;
    const int dir = (p.eend[2 * e2] == a) ? 1 : 0;    // the message travelling towards a
    return reinterpret_cast<const cpx<S>*>(p.msg) + ((size_t)e2 * 2 + dir) * CHI * CHI;
}

__device__ __forceinline__ double leg_lambda(const DevPool& p, int a, int l, int j, int CHI) {
    const int e2 = p.vedge[3 * a + l];
    if (e2 < 0) return j == 0 ? 1.0 : 0.0;
    return p.lam[(size_t)e2 * CHI + j];
}

}  // namespace gtqa
