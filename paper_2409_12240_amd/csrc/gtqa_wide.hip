// HIP kernels (gfx950) of the GTQA Trotter step at bond dimension chi = 16.
//
// At chi = 16 a site tensor holds 2 x 16^3 complex values (64 KB in complex64),
// the BP message update and the gauge application are three mode products of
// 2 chi^4 complex multiply-adds each, and the simple update's blocks are
// 256 x 16.  The contractions run on the matrix cores (MFMA 16x16x4, FP32 for
// complex64 storage, FP64 for complex128), the bond QR and SVD in FP64 on the
// vector units.
//
//   k16_bp_class      one colour class of a BP sweep (Alg. 1): four wavefronts
//                     per edge, one per (direction, physical index); the three
//                     products of Eq. local_consistency as 16x16 MFMA tiles.
//   k16_gauge_apply   Alg. 2's gauge maps on the three legs (MFMA), U_X fused.
//   k16_su_qr         simple update (App. E), stage 1: Householder QR of one
//                     256 x 16 physical block per wavefront; reflectors, R
//                     and their scales go to a workspace.
//   k16_su_core       stage 2: the 32 x 32 bond core with the gate phases,
//                     one-sided Jacobi SVD, truncation to chi (Alg. 3), lambda,
//                     fidelity and truncation error, the kept singular vectors.
//   k16_su_apply      stage 3: Q times the kept vectors, divided by the outer
//                     lambdas, written as the new Gamma.
//   k16_canonicalise  Alg. 2 per edge in FP64 (factor, core SVD, gauge maps).
//
// MFMA 16x16x4 lane layout (wave64; lane L = 16 g + n, g < 4, n < 16): the A
// operand is A[n][g], the B operand B[g][n], and accumulator register r holds
// D[row(g, r)][n] with row(g, r) = 4 g + r for the FP32 instruction and
// g + 4 r for the FP64 one (measured).  A 16x16 accumulator tile therefore
// serves directly as the A operand of the next product over its row index
// (register r is the chunk whose K-value in lane group g is row(g, r)), which
// is how consecutive mode products chain without data movement; every chunk
// of K-values uses the same map, and one 4 x 4 block transpose across the
// lane groups (two xor exchanges) moves the contracted index where it is
// needed.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gtqa.h"
#include "gtqa_internal.h"
#include "gtqa_device.h"

namespace gtqa {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename S>
struct Mfma;
template <>
struct Mfma<float> {
    using acc = f32x4;
    __device__ static acc run(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
};
template <>
struct Mfma<double> {
    using acc = f64x4;
    __device__ static acc run(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
};

// row of accumulator register r in lane group g (see above); also the
// K-value that lane group g supplies in chunk r
template <typename S>
__device__ __forceinline__ constexpr int mrow(int g, int r) {
    return sizeof(S) == 4 ? 4 * g + r : g + 4 * r;
}

// complex 16x16 accumulator tile
template <typename S>
struct CTile {
    typename Mfma<S>::acc re, im;
};
template <typename S>
__device__ __forceinline__ CTile<S> ctile_zero() {
    return {Mfma<S>::zero(), Mfma<S>::zero()};
}
// D += A B (one K-chunk of 4), complex A and B; nai = -A.im
template <typename S>
__device__ __forceinline__ void cmfma(CTile<S>& d, S ar, S ai, S nai, S br, S bi) {
    d.re = Mfma<S>::run(ar, br, d.re);
    d.re = Mfma<S>::run(nai, bi, d.re);
    d.im = Mfma<S>::run(ar, bi, d.im);
    d.im = Mfma<S>::run(ai, br, d.im);
}

// value of lane ^ MASK (MASK 16 or 32 here)
template <int MASK>
__device__ __forceinline__ float lane_xor(float v) { return __int_as_float(xshfl_i(__float_as_int(v), MASK)); }
template <int MASK>
__device__ __forceinline__ double lane_xor(double v) { return xshfl(v, MASK); }

// 4 x 4 block transpose across the lane groups g = lane / 16.  v[mrow(s, q)][r]
// (s, q, r < 4) is slot s of the lane; afterwards slot s of lane group c holds
// what slot c of lane group s held (same q, r), for every n = lane % 16.
// Two xor exchanges: lane bit 5 (group bit 1), then lane bit 4 (group bit 0).
template <typename S>
__device__ __forceinline__ void group_transpose(cpx<S> (&v)[16][4], int g) {
    {
        const bool b = (g >> 1) & 1;
#pragma unroll
        for (int s0 = 0; s0 < 2; ++s0)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ia = mrow<S>(s0, q), ib = mrow<S>(s0 + 2, q);
                    const cpx<S> A = v[ia][r];
                    const cpx<S> B = v[ib][r];
                    const cpx<S> send = b ? A : B;
                    const cpx<S> recv = {lane_xor<32>(send.re), lane_xor<32>(send.im)};
                    v[ia][r] = b ? recv : A;
                    v[ib][r] = b ? B : recv;
                }
    }
    {
        const bool b = g & 1;
#pragma unroll
        for (int s0 = 0; s0 < 4; s0 += 2)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ia = mrow<S>(s0, q), ib = mrow<S>(s0 + 1, q);
                    const cpx<S> A = v[ia][r];
                    const cpx<S> B = v[ib][r];
                    const cpx<S> send = b ? A : B;
                    const cpx<S> recv = {lane_xor<16>(send.re), lane_xor<16>(send.im)};
                    v[ia][r] = b ? recv : A;
                    v[ib][r] = b ? B : recv;
                }
    }
}

template <typename S>
__device__ __forceinline__ void tile_to_regs(const CTile<S>& t, cpx<S> (&o)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = {t.re[r], t.im[r]};
}

// ------------------------------------------------------------------ BP (chi = 16)
// m_out[j][j'] = sum T[i, j@p, k@o1, l@o2] conj(T[i, j'@p, k'@o1, l'@o2]) m1[k][k'] m2[l][l']
// with T = Gamma prod sqrt(lambda).  The square roots of the o1, o2 lambdas
// are folded into the incoming messages (m~[k][k'] = sqrt(l_k) m[k][k'] sqrt(l_k')),
// those of the outgoing leg into the result, so Gamma is read as stored.
// Per (direction, i), with j on the lane (n) and the contracted indices
// spread over lane groups and registers:
//   1. Y[j][k'][l] = sum_k m1~[k][k'] Gamma[i][j][k][l]   16 tiles (l), rows k'
//   2. block transpose: lane group c then holds l = mrow(c, q) for every k'
//   3. Z[j][k'][l'] = sum_l m2~[l][l'] Y[j][k'][l]        16 tiles (k'), rows l'
//   4. out[j][j'] += sum_{k', l'} Z[j][k'][l'] conj(Gamma[i][j'][k'][l'])
// The two physical halves i run in two wavefronts and are summed in LDS.
// In FP32 the kernel fits 256 registers without spilling, so it runs two
// wavefronts per SIMD (769 -> 662 us per launch of 6000 edges, measured);
// the FP64 instantiation would spill there and keeps one.
// WARM (with FIRST): both incoming messages are diagonal (the first class of
// a first sweep: every neighbouring edge belongs to a later class; every
// class of a flooding first sweep), so steps 1-3 reduce to
// Z[j][k'][l'] = (Gamma[i][j][k'][l'] m1~[k'][k']) m2~[l'][l'], the values
// the two products give (their off-diagonal terms add exact zeros), formed
// from the Gamma entries step 4 loads anyway.
template <int CHI, typename S, bool FIRST, bool FLOOD, bool WARM = false>
__global__ __launch_bounds__(256, sizeof(S) == 4 ? 2 : 1) void k16_bp_class(DevPool p, const int4* recs,
                                                                           int nitems, int cls,
                                                                           const int32_t* gate) {
    static_assert(CHI == 16, "chi = 16 layout");
    static_assert(!WARM || FIRST, "warm-start messages exist only in a first sweep");
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int M2 = CHI * CHI;
    using W = cpx<S>;
    __shared__ double lamv[2][3][CHI];
    __shared__ W mt[2][2][M2];               // scaled incoming messages per direction
    __shared__ W half1[2][M2];               // physical half i = 1 of each direction's result
    __shared__ double bnd[2][2];

    const int item = wg_index(p.xcd_remap);
    if (item >= nitems) return;              // uniform
    if (gate && *gate == 0) return;          // uniform
    const int4* rec = recs + 3 * (size_t)item;
    const int4 es = rec[2];
    const int e = es.x, slot = es.y;
    const int fl = p.sflag[slot];
    // one edge per work-group: the flag is uniform
    if (!(fl & FLAG_ACTIVE) || (fl & (FLAG_BP_DONE | FLAG_UNDECIDED))) return;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    const int d = w >> 1, ih = w & 1;
    const int g = lane >> 4, n = lane & 15;
    const int4 md = rec[d];
    const int pleg = md.w & 3;
    int o1, o2;
    other_legs(pleg, o1, o2);

    if (tid < 2 * 3 * CHI) {
        const int dd = tid / (3 * CHI), lg = (tid / CHI) % 3, j = tid % CHI;
        const int4 mdd = rec[dd];
        const int pl = mdd.w & 3;
        int q1, q2;
        other_legs(pl, q1, q2);
        const int inc = lg == pl ? 2 * e : (lg == q1 ? mdd.y : mdd.z);
        lamv[dd][lg][j] = inc >= 0 ? p.lam[(size_t)(inc >> 1) * CHI + j] : (j == 0 ? 1.0 : 0.0);
    }
    __syncthreads();
    // incoming messages, sqrt(lambda) on both indices; missing legs e0 e0^T,
    // in the first sweep those of classes not yet visited (flooding: all)
    // the warm start diag(lambda)/sum(lambda); flooding reads the previous
    // iterate from mold
    for (int idx = tid; idx < 2 * 2 * M2; idx += 256) {
        const int dd = idx / (2 * M2), ww = (idx / M2) & 1, o = idx % M2;
        const int4 mdd = rec[dd];
        const int pl = mdd.w & 3;
        int q1, q2;
        other_legs(pl, q1, q2);
        const int lg = ww == 0 ? q1 : q2;
        const int inc = ww == 0 ? mdd.y : mdd.z;
        const int col = (mdd.w >> (8 + 8 * ww)) & 255;
        const int r = o / CHI, c = o % CHI;
        cd val;
        if (inc < 0) {
            val = {o == 0 ? 1.0 : 0.0, 0.0};
        } else if (FIRST && (FLOOD || col > cls)) {
            double tot = 0.0;
            for (int j = 0; j < CHI; ++j) tot += lamv[dd][lg][j];
            val = {(r == c && tot > 0.0) ? lamv[dd][lg][r] / tot : 0.0, 0.0};
        } else {
            val = to_cd(reinterpret_cast<const W*>(FLOOD ? p.mold : p.msg)[(size_t)inc * M2 + o]);
        }
        const double sc = sqrt(lamv[dd][lg][r]) * sqrt(lamv[dd][lg][c]);
        mt[dd][ww][o] = from_cd<S>(cscale(val, sc));
    }
    __syncthreads();

    const int sp = leg_stride<CHI>(pleg), s1 = leg_stride<CHI>(o1), s2 = leg_stride<CHI>(o2);
    const W* gam = reinterpret_cast<const W*>(p.gam) + (size_t)md.x * 2 * C3 + (size_t)ih * C3;
    CTile<S> acc = ctile_zero<S>();
    if constexpr (WARM) {
        const W* gb = gam + n * sp;
#pragma unroll
        for (int kp = 0; kp < CHI; ++kp) {
            const S d1 = mt[d][0][kp * CHI + kp].re;
#pragma unroll
            for (int r2 = 0; r2 < 4; ++r2) {
                const int lq = mrow<S>(g, r2);
                const W tv = gb[kp * s1 + lq * s2];
                const S d2 = mt[d][1][lq * CHI + lq].re;
                const S zr = (tv.re * d1) * d2, zi = (tv.im * d1) * d2;
                acc.re = Mfma<S>::run(zr, tv.re, acc.re);
                acc.re = Mfma<S>::run(zi, tv.im, acc.re);
                acc.im = Mfma<S>::run(-zr, tv.im, acc.im);
                acc.im = Mfma<S>::run(zi, tv.re, acc.im);
            }
        }
    } else {
    // A operands: chunk kk holds K-values mrow(g, kk)
    W a1[4], a2[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        a1[kk] = mt[d][0][mrow<S>(g, kk) * CHI + n];
        a2[kk] = mt[d][1][mrow<S>(g, kk) * CHI + n];
    }
    // 1. Y tiles (one per l): lane (g, n), register r = Y[j = n][k' = mrow(g, r)][l]
    W y[16][4];
    {
        const W* gb = gam + n * sp;
#pragma unroll
        for (int l = 0; l < CHI; ++l) {
            CTile<S> t = ctile_zero<S>();
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const W b = gb[mrow<S>(g, kk) * s1 + l * s2];
                cmfma<S>(t, a1[kk].re, a1[kk].im, -a1[kk].im, b.re, b.im);
            }
            tile_to_regs<S>(t, y[l]);
        }
    }
    // 2. now y[mrow(s, q)][r] = Y[n][k' = mrow(s, r)][l = mrow(g, q)]
    group_transpose<S>(y, g);
    // 3.-4. per k' = mrow(s, r): Z tile, then its contribution to the result
    {
        const W* gb = gam + n * sp;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int kp = mrow<S>(s, r);
                CTile<S> t = ctile_zero<S>();
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const W b = y[mrow<S>(s, kk)][r];
                    cmfma<S>(t, a2[kk].re, a2[kk].im, -a2[kk].im, b.re, b.im);
                }
                // lane (g, n), register r2 = Z[j = n][k'][l' = mrow(g, r2)]: the A
                // operand of chunk r2 (K-values (k', mrow(g, r2))) of the last product
#pragma unroll
                for (int r2 = 0; r2 < 4; ++r2) {
                    const W tv = gb[kp * s1 + mrow<S>(g, r2) * s2];
                    const S zr = t.re[r2], zi = t.im[r2];
                    // A = Z, B = conj(Gamma)
                    acc.re = Mfma<S>::run(zr, tv.re, acc.re);
                    acc.re = Mfma<S>::run(zi, tv.im, acc.re);
                    acc.im = Mfma<S>::run(-zr, tv.im, acc.im);
                    acc.im = Mfma<S>::run(zi, tv.re, acc.im);
                }
            }
    }
    }
    // acc register r = out~_i[j = mrow(g, r)][j' = n]
    if (ih == 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) half1[d][mrow<S>(g, r) * CHI + n] = {acc.re[r], acc.im[r]};
    }
    __syncthreads();
    double fro = 0.0, hi = 0.0;
    if (ih == 0) {
        cd tot[4];
        const double sqn = sqrt(lamv[d][pleg][n]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = mrow<S>(g, r);
            const cd h = to_cd(half1[d][j * CHI + n]);
            const cd s0 = {double(acc.re[r]) + h.re, double(acc.im[r]) + h.im};
            tot[r] = cscale(s0, sqrt(lamv[d][pleg][j]) * sqn);
        }
        // unit trace by the complex trace
        cd tr = cz<double>();
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (mrow<S>(g, r) == n) tr = cadd(tr, tot[r]);
        tr = seg_sum<64>(tr);
        const double t2 = cabs2(tr);
        const double it2 = t2 > 0.0 ? 1.0 / t2 : 0.0;
        const cd itr = {tr.re * it2, -tr.im * it2};
        W* dst = reinterpret_cast<W*>(p.msg) + ((size_t)e * 2 + d) * M2;
        W* mo = reinterpret_cast<W*>(p.mold) + ((size_t)e * 2 + d) * M2;
        double lt = 0.0;
        if (FIRST)
            for (int j = 0; j < CHI; ++j) lt += lamv[d][pleg][j];
        double f2 = 0.0, l1 = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = mrow<S>(g, r);
            const int o = j * CHI + n;
            W oldv;
            if (FIRST) oldv = {S((j == n && lt > 0.0) ? lamv[d][pleg][j] / lt : 0.0), S(0)};
            else oldv = FLOOD ? mo[o] : dst[o];
            const W nvs = from_cd<S>(cmul(tot[r], itr));
            const cd df = csub(to_cd(nvs), to_cd(oldv));
            dst[o] = nvs;
            if (!FLOOD || FIRST) mo[o] = oldv;
            const double a2v = cabs2(df);
            f2 += a2v;
            l1 += sqrt(a2v);
        }
        f2 = seg_sum<64>(f2);
        l1 = seg_sum<64>(l1);
        fro = sqrt(f2);
        hi = fmin(sqrt((double)CHI) * fro, l1);
        if (lane == 0) {
            bnd[d][0] = fro;
            bnd[d][1] = hi;
        }
    }
    __syncthreads();
    if (tid == 0) {
        p.edlo[e] = bnd[0][0] + bnd[1][0];
        p.edist[e] = bnd[0][1] + bnd[1][1];
    }
}

// ------------------------------------------------------------------ gauge apply (chi = 16)
// Gamma[i][a'][b'][c'] = sum_{a,b,c} T[i][a][b][c] X0[a][a'] X1[b][b'] X2[c][c'],
// T = Gamma_old (the sqrt(lambda_old) are folded into the maps), with U_X
// (which acts on i only and commutes with the maps) applied as the tensor is
// read.  One wavefront per physical half i:
//   1. G1[a][b][c'] = sum_c T[a][b][c] X2[c][c']   16 tiles (a), rows b
//   2. G2[a][b'][c'] = sum_b G1[a][b][c'] X1[b][b'] same tiles, rows c' (the
//      accumulator of 1. is the A operand over its row index b)
//   3. block transpose: lane group c then holds a = mrow(c, q) for every c'
//   4. G3[a'][b'][c'] = sum_a G2[a][b'][c'] X0[a][a']  16 tiles (c'), rows b'
// Two wavefronts per SIMD in FP32 (172 registers, no spills: 1165 -> 897 us
// per launch of 16,000 vertices, measured); one in FP64.
template <int CHI, typename S>
__global__ __launch_bounds__(128, sizeof(S) == 4 ? 2 : 1) void k16_gauge_apply(DevPool p, const int32_t* items,
                                                                              int nitems, int apply_x_allowed) {
    if (tail_gated_off(p)) return;       // uniform: BP has not stopped
    static_assert(CHI == 16, "chi = 16 layout");
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int M2 = CHI * CHI;
    using W = cpx<S>;
    const int item = wg_index(p.xcd_remap);
    if (item >= nitems) return;
    const int a = items[item];
    const int4 vm = p.vmeta[a];
    const int slot = vm.w;
    const int fl = p.sflag[slot];
    if (!(fl & FLAG_ACTIVE)) return;          // uniform
    const int ih = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, n = lane & 15;
    const W* xg = reinterpret_cast<const W*>(p.xg);
    auto xmap = [&](int lg, int row, int col) -> W {
        const int xi = lg == 0 ? vm.x : (lg == 1 ? vm.y : vm.z);
        if (xi < 0) return {S(row == 0 && col == 0 ? 1 : 0), S(0)};
        return xg[(size_t)xi * M2 + row * CHI + col];
    };
    // B operands: chunk kk holds rows mrow(g, kk)
    W x0[4], x1[4], x2[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        x0[kk] = xmap(0, mrow<S>(g, kk), n);
        x1[kk] = xmap(1, mrow<S>(g, kk), n);
        x2[kk] = xmap(2, mrow<S>(g, kk), n);
    }
    const bool do_x = apply_x_allowed && (fl & FLAG_APPLY_X);
    S cx = S(1), sx = S(0);
    if (do_x) {
        double sn, cs;
        sincos(p.theta[2 * slot + 1], &sn, &cs);
        cx = S(cs);
        sx = S(sn);
    }
    W* gam = reinterpret_cast<W*>(p.gam) + (size_t)a * 2 * C3;
    const W* gi = gam + (size_t)ih * C3;
    const W* go = gam + (size_t)(1 - ih) * C3;
    // 1.-2. per a: lane (g, n) register r = G2[a][b' = n][c' = mrow(g, r)]
    W v[16][4];
#pragma unroll
    for (int aa = 0; aa < CHI; ++aa) {
        CTile<S> t = ctile_zero<S>();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            // A[b = n][c = mrow(g, kk)] = T[a][n][mrow(g, kk)], U_X mixed in:
            // [c, -i s; -i s, c] on the physical index
            const int o = aa * M2 + n * CHI + mrow<S>(g, kk);
            const W t0 = gi[o];
            W av = t0;
            if (do_x) {
                const W t1 = go[o];
                av = {cx * t0.re + sx * t1.im, cx * t0.im - sx * t1.re};
            }
            cmfma<S>(t, av.re, av.im, -av.im, x2[kk].re, x2[kk].im);
        }
        // t register r = G1[a][b = mrow(g, r)][c' = n]: chunk r of the next product
        CTile<S> u = ctile_zero<S>();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const S ar = t.re[r], ai = t.im[r];
            cmfma<S>(u, ar, ai, -ai, x1[r].re, x1[r].im);
        }
        tile_to_regs<S>(u, v[aa]);
    }
    __syncthreads();                          // both halves read before either is written
    // 3. now v[mrow(s, q)][r] = G2[a = mrow(g, q)][b' = n][c' = mrow(s, r)]
    group_transpose<S>(v, g);
    // 4. per c' = mrow(s, r); the tile's result replaces the four registers
    // it consumed: v[mrow(s, r3)][r] = G3[a' = n][b' = mrow(g, r3)][c' = mrow(s, r)]
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            CTile<S> t = ctile_zero<S>();
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const W av = v[mrow<S>(s, kk)][r];
                cmfma<S>(t, av.re, av.im, -av.im, x0[kk].re, x0[kk].im);
            }
#pragma unroll
            for (int r3 = 0; r3 < 4; ++r3) v[mrow<S>(s, r3)][r] = {t.re[r3], t.im[r3]};
        }
    // each lane now holds, for each r3, the whole row (a' = n, b' = mrow(g, r3))
    // over c': 16 contiguous values, written as 16-byte vectors
    W* gw = gam + (size_t)ih * C3;
#pragma unroll
    for (int r3 = 0; r3 < 4; ++r3) {
        W* row = gw + n * M2 + mrow<S>(g, r3) * CHI;
        W vals[CHI];
#pragma unroll
        for (int cp = 0; cp < CHI; ++cp) {
            const int sc = sizeof(S) == 4 ? cp >> 2 : cp & 3;
            const int rc = sizeof(S) == 4 ? cp & 3 : cp >> 2;
            vals[cp] = v[mrow<S>(sc, r3)][rc];
        }
        if constexpr (sizeof(S) == 4) {
            float4* dst = reinterpret_cast<float4*>(row);
#pragma unroll
            for (int c2 = 0; c2 < CHI / 2; ++c2)
                dst[c2] = make_float4(vals[2 * c2].re, vals[2 * c2].im, vals[2 * c2 + 1].re, vals[2 * c2 + 1].im);
        } else {
#pragma unroll
            for (int cp = 0; cp < CHI; ++cp) row[cp] = vals[cp];
        }
    }
}

// ------------------------------------------------------------------ simple update (chi = 16)
// Workspace layout per edge of a chunk (doubles): the four blocks' QR data
// [4][chi cols][chi^2 rows] complex (column-major, so a wavefront's rows are
// contiguous), R factors [4][chi][chi] complex, reflector scales [4][chi],
// kept vectors Z [4][chi][chi] complex.
template <int CHI>
struct SuWs {
    static constexpr int ROWS = CHI * CHI;
    static constexpr size_t H = (size_t)4 * CHI * ROWS * 2;
    static constexpr size_t R = (size_t)4 * CHI * CHI * 2;
    static constexpr size_t V = (size_t)4 * CHI;
    static constexpr size_t Z = (size_t)4 * CHI * CHI * 2;
    static constexpr size_t PER_EDGE = H + R + V + Z;
    __device__ static double* h(double* ws, int ci, int b) { return ws + (size_t)ci * PER_EDGE + (size_t)b * CHI * ROWS * 2; }
    __device__ static double* r(double* ws, int ci, int b) { return ws + (size_t)ci * PER_EDGE + H + (size_t)b * CHI * CHI * 2; }
    __device__ static double* v(double* ws, int ci, int b) { return ws + (size_t)ci * PER_EDGE + H + R + (size_t)b * CHI; }
    __device__ static double* z(double* ws, int ci, int b) { return ws + (size_t)ci * PER_EDGE + H + R + V + (size_t)b * CHI * CHI * 2; }
};

size_t su_ws_bytes_per_edge(int chi) {
    return chi == 16 ? SuWs<16>::PER_EDGE * sizeof(double) : 0;
}

// Sum of each of v[0..NV) over the 64 lanes of the wavefront, in every lane
// (NV a power of two, at most 64).  Recursive halving: at the level with lane
// mask M a lane keeps the upper half of its values if its lane has bit M
// set (else the lower), adds its partner's copy of that half and sends the
// other half; after log2(NV) levels each lane holds one partial sum, the
// remaining lane bits are summed by a butterfly, and recursive doubling (the
// levels in reverse, copies only) returns every sum to every lane, bitwise
// the same in all of them.  2 (NV - 1) + log2(64 / NV) exchanged values
// instead of 6 NV for NV separate butterflies.
template <int SZ, int M>
__device__ __forceinline__ void wr_halve(double* v, int lane) {
    const bool up = (lane & M) != 0;
#pragma unroll
    for (int i = 0; i < SZ / 2; ++i) {
        const double lo = v[i], hi = v[i + SZ / 2];
        const double send = up ? lo : hi;
        const double keep = up ? hi : lo;
        v[i] = keep + xshfl(send, M);
    }
}
template <int SZ, int M>
__device__ __forceinline__ void wr_double(double* v, int lane) {
    const bool up = (lane & M) != 0;
#pragma unroll
    for (int i = 0; i < SZ; ++i) {
        const double mine = v[i];
        const double other = xshfl(mine, M);
        v[i] = up ? other : mine;
        v[i + SZ] = up ? mine : other;
    }
}
template <int NV>
__device__ __forceinline__ void wave_allreduce(double (&v)[NV], int lane) {
    static_assert(NV == 16, "the chi = 16 kernels reduce 8 complex values at a time");
    wr_halve<16, 32>(v, lane);
    wr_halve<8, 16>(v, lane);
    wr_halve<4, 8>(v, lane);
    wr_halve<2, 4>(v, lane);
    v[0] += xshfl(v[0], 2);
    v[0] += xshfl(v[0], 1);
    wr_double<1, 4>(v, lane);
    wr_double<2, 8>(v, lane);
    wr_double<4, 16>(v, lane);
    wr_double<8, 32>(v, lane);
}

__device__ __forceinline__ double readlane_d(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Block b of edge items[ci]: b = 0, 1 -> Gamma_u[i = b] with the outer lambdas
// of u on its rows and lambda_e on its columns; b = 2, 3 -> Gamma_v[i = b - 2]
// with the outer lambdas of v.  Rows (j1, j2) of the two outer legs, column
// the bond leg; lane t holds rows t + 64 k.
template <int CHI>
__device__ __forceinline__ void su_block_geometry(const DevPool& p, int e, int b, int& vert, int& pleg, int& o1,
                                                  int& o2) {
    const int side = b >> 1;
    vert = p.eend[2 * e + side];
    pleg = p.eleg[2 * e + side];
    other_legs(pleg, o1, o2);
}

template <int CHI, typename S>
__global__ __launch_bounds__(64) void k16_su_qr(DevPool p, const int32_t* items, int nc) {
    static_assert(CHI == 16, "chi = 16 layout");
    constexpr int ROWS = CHI * CHI;
    constexpr int RPL = ROWS / 64;
    constexpr int C3 = CHI * CHI * CHI;
    __shared__ double lamv[3][CHI];
    __shared__ double lame[CHI];
    const int b = blockIdx.x & 3, ci = blockIdx.x >> 2;
    if (ci >= nc) return;
    const int e = items[ci];
    const int lane = threadIdx.x;
    const int side = b >> 1, ib = b & 1;
    int vert, pleg, o1, o2;
    su_block_geometry<CHI>(p, e, b, vert, pleg, o1, o2);
    if (lane < 3 * CHI) lamv[lane / CHI][lane % CHI] = leg_lambda(p, vert, lane / CHI, lane % CHI, CHI);
    if (lane < CHI) lame[lane] = side == 0 ? p.lam[(size_t)e * CHI + lane] : 1.0;
    __syncthreads();
    const int s1 = leg_stride<CHI>(o1), s2 = leg_stride<CHI>(o2), sp = leg_stride<CHI>(pleg);
    const cpx<S>* gsrc = reinterpret_cast<const cpx<S>*>(p.gam) + (size_t)vert * 2 * C3 + (size_t)ib * C3;
    cd xr[RPL][CHI];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int row = lane + 64 * k;
        const int j1 = row / CHI, j2 = row % CHI;
        const double sc = lamv[o1][j1] * lamv[o2][j2];
#pragma unroll
        for (int j = 0; j < CHI; ++j) xr[k][j] = cscale(to_cd(gsrc[j1 * s1 + j2 * s2 + j * sp]), sc * lame[j]);
    }
    // Householder QR: reflector kc = (top, x[kc+1:, kc]) in place, top in
    // row kc (lane kc, k = 0), 2/|v|^2 in v2 (0: no reflection)
    cd rdiag = cz<double>();
    double v2[CHI];
#pragma unroll
    for (int kc = 0; kc < CHI; ++kc) {
        double part = 0.0;
#pragma unroll
        for (int k = 0; k < RPL; ++k)
            if (k > 0 || lane >= kc) part += cabs2(xr[k][kc]);
        const double nrm2 = seg_sum<64>(part);
        const cd alpha = {readlane_d(xr[0][kc].re, kc), readlane_d(xr[0][kc].im, kc)};
        const double nrm = sqrt(nrm2);
        const double aa = sqrt(cabs2(alpha));
        if (nrm > 0.0) {
            const cd ph = aa > 0.0 ? cd{alpha.re / aa, alpha.im / aa} : cd{1.0, 0.0};
            const cd top = {alpha.re + ph.re * nrm, alpha.im + ph.im * nrm};
            v2[kc] = 2.0 / (2.0 * nrm * (nrm + aa));
            cd vk[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k)
                vk[k] = (k > 0 || lane > kc) ? xr[k][kc] : (lane == kc ? top : cz<double>());
#pragma unroll
            for (int jc = kc + 1; jc < CHI; ++jc) {
                cd w = cz<double>();
#pragma unroll
                for (int k = 0; k < RPL; ++k) w = ccfma(w, vk[k], xr[k][jc]);
                w = seg_sum<64>(w);
                const cd f = cscale(w, v2[kc]);
#pragma unroll
                for (int k = 0; k < RPL; ++k) xr[k][jc] = csub(xr[k][jc], cmul(f, vk[k]));
            }
            if (lane == kc) {
                rdiag = {-ph.re * nrm, -ph.im * nrm};
                xr[0][kc] = top;
            }
        } else {
            v2[kc] = 0.0;
        }
    }
    double* H = SuWs<CHI>::h(p.su_ws, ci, b);
#pragma unroll
    for (int j = 0; j < CHI; ++j)
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const size_t o = ((size_t)j * ROWS + lane + 64 * k) * 2;
            H[o] = xr[k][j].re;
            H[o + 1] = xr[k][j].im;
        }
    double* Rw = SuWs<CHI>::r(p.su_ws, ci, b);
    if (lane < CHI) {
#pragma unroll
        for (int j = 0; j < CHI; ++j) {
            const cd v = j > lane ? xr[0][j] : (j == lane ? rdiag : cz<double>());
            Rw[(lane * CHI + j) * 2] = v.re;
            Rw[(lane * CHI + j) * 2 + 1] = v.im;
        }
    }
    if (lane < CHI) {
        double vv = 0.0;
#pragma unroll
        for (int kc = 0; kc < CHI; ++kc) vv = lane == kc ? v2[kc] : vv;
        SuWs<CHI>::v(p.su_ws, ci, b)[lane] = vv;
    }
}

// The bond core M[(iu, pa)][(iv, qb)] = phi(iu, iv) sum_k R_u,iu[pa][k] R_v,iv[qb][k],
// its SVD (columns presorted by norm, one-sided Jacobi in FP64), truncation
// to the chi largest values above the cutoff, lambda_e, log f and eps, and
// the kept vectors: U rows for the u blocks, conj(V) rows for the v blocks.
// V is recovered as M^dagger U from the R factors,
// V[(iv, qb)][q] = sum_iu conj(phi(iu, iv)) sum_k conj(R_v,iv[qb][k]) W_iu[k][q],
// W_iu[k][q] = sum_pa conj(R_u,iu[pa][k]) U[(iu, pa)][q],
// and orthonormalised by two Gram-Schmidt passes.  LDS holds one 16 KB
// buffer (the R factors, later U and V), so eight cores fit a CU.
template <int CHI, typename S>
__global__ __launch_bounds__(64, 2) void k16_su_core(DevPool p, const int32_t* items, int nc) {
    static_assert(CHI == 16, "chi = 16 layout");
    constexpr int N = 2 * CHI;
    constexpr int LPC = JLayout<N, 64>::LPC;
    constexpr int EPL = JLayout<N, 64>::EPL;
    __shared__ cd buf[4 * CHI * CHI];
    cd (*Rl)[CHI][CHI] = reinterpret_cast<cd (*)[CHI][CHI]>(buf);
    cd (*Ul)[CHI] = reinterpret_cast<cd (*)[CHI]>(buf);              // [N][CHI], kept columns by rank
    cd (*Vl)[CHI] = reinterpret_cast<cd (*)[CHI]>(buf + N * CHI);    // [N][CHI]
    __shared__ cd phl[2][2];
    __shared__ double sig[N];
    __shared__ int order[N];
    const int ci = blockIdx.x;
    if (ci >= nc) return;
    const int e = items[ci];
    const int el = threadIdx.x;
    const int slot = p.eslot[e];
    const double theta = p.theta[2 * slot];
    for (int idx = el; idx < 4 * CHI * CHI; idx += 64) {
        const int b = idx / (CHI * CHI), o = idx % (CHI * CHI);
        const double* src = SuWs<CHI>::r(p.su_ws, ci, b) + 2 * o;
        Rl[b][o / CHI][o % CHI] = {src[0], src[1]};
    }
    if (el < 4) {
        const int iu = el >> 1, iv = el & 1;
        const double zu = iu ? -1.0 : 1.0, zv = iv ? -1.0 : 1.0;
        const double ang = -theta * (p.J[e] * zu * zv + p.hD[p.eend[2 * e]] * zu + p.hD[p.eend[2 * e + 1]] * zv);
        double sn, cs;
        sincos(ang, &sn, &cs);
        phl[iu][iv] = {cs, sn};
    }
    __syncthreads();
    const int ccol = JLayout<N, 64>::col(el);
    const int cg = JLayout<N, 64>::grp(el);
    cd m[EPL], v[1];
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int row = cg + LPC * k;
        const int iu = row / CHI, pa = row % CHI;
        const int iv = ccol / CHI, qb = ccol % CHI;
        cd acc = cz<double>();
#pragma unroll
        for (int kk = 0; kk < CHI; ++kk) acc = cfma(acc, Rl[iu][pa][kk], Rl[2 + iv][qb][kk]);
        m[k] = cmul(acc, phl[iu][iv]);
    }
    // columns presorted by norm (descending, ties by index): position c takes
    // the column of rank c from its lane in the same row group
    {
        double own2 = 0.0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) own2 += cabs2(m[k]);
        own2 = strided_sum<N, LPC>(own2);
        if (cg == 0) sig[ccol] = own2;
        __syncthreads();
        int rk = 0;
        const double me = sig[ccol];
        for (int c = 0; c < N; ++c) {
            const double o = sig[c];
            rk += (o > me || (o == me && c < ccol)) ? 1 : 0;
        }
        if (cg == 0) order[rk] = ccol;
        __syncthreads();
        const int src = order[ccol] + N * cg;
#pragma unroll
        for (int k = 0; k < EPL; ++k) m[k] = {__shfl(m[k].re, src, 64), __shfl(m[k].im, src, 64)};
        __syncthreads();                     // sig and order are reused below
    }
    const int sweeps = jacobi_svd_team<N, 64, false, N, true>(m, v, el, JACOBI_TOL, JACOBI_MAX_SWEEPS);
    if (sweeps > JACOBI_MAX_SWEEPS && el == 0) atomicOr(&p.swarn[slot], (int)WARN_JACOBI);
    double nrm_loc = 0.0;
#pragma unroll
    for (int k = 0; k < EPL; ++k) nrm_loc += cabs2(m[k]);
    nrm_loc = strided_sum<N, LPC>(nrm_loc);
    const double sgm = sqrt(nrm_loc);
    if (cg == 0) sig[ccol] = sgm;
    __syncthreads();
    int myrank = 0;
    {
        for (int c = 0; c < N; ++c) {
            const double o = sig[c];
            myrank += (o > sgm || (o == sgm && c < ccol)) ? 1 : 0;
        }
        if (cg == 0 && myrank < N) order[myrank] = ccol;
    }
    __syncthreads();
    const double smax = sig[order[0]];
    int r = 0;
    double kept2 = 0.0;
    for (int k = 0; k < CHI; ++k) {
        const double sk = sig[order[k]];
        if (sk > p.svd_cut * smax) {
            r = k + 1;
            kept2 += sk * sk;
        }
    }
    const double inv_norm = kept2 > 0.0 ? 1.0 / sqrt(kept2) : 0.0;
    if (el == 0) {
        double tot = 0.0, dropped = 0.0;
        for (int k = 0; k < N; ++k) {
            const double sk = sig[order[k]];
            tot += sk * sk;
            if (k >= r) dropped += sk * sk;
        }
        p.elogf[e] = tot > 0.0 ? 2.0 * log(kept2 / tot) : 0.0;
        p.eeps[e] = tot > 0.0 ? sqrt(dropped / tot) : 0.0;
        p.efix[e] = 0;
    }
    if (el < CHI) p.lam[(size_t)e * CHI + el] = el < r ? sig[order[el]] * inv_norm : 0.0;
    // kept U columns by rank (zero from rank r on); the R factors are no
    // longer read from LDS
    if (myrank < CHI) {
        const double isg = (myrank < r && sgm > 0.0) ? 1.0 / sgm : 0.0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) Ul[cg + LPC * k][myrank] = cscale(m[k], isg);
    }
    __syncthreads();
    const double* Ru[2] = {SuWs<CHI>::r(p.su_ws, ci, 0), SuWs<CHI>::r(p.su_ws, ci, 1)};
    const double* Rv[2] = {SuWs<CHI>::r(p.su_ws, ci, 2), SuWs<CHI>::r(p.su_ws, ci, 3)};
    // W_iu[k][q] into the V buffer
    {
        cd wv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int idx = el + 64 * j;
            const int iu = idx / (CHI * CHI), kk = (idx / CHI) % CHI, q = idx % CHI;
            cd acc = cz<double>();
            for (int pa = 0; pa < CHI; ++pa) {
                const double* a = Ru[iu] + 2 * (pa * CHI + kk);
                acc = ccfma(acc, cd{a[0], a[1]}, Ul[iu * CHI + pa][q]);
            }
            wv[j] = acc;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int idx = el + 64 * j;
            Vl[idx / CHI][idx % CHI] = wv[j];       // W_iu[k][q] at row iu chi + k
        }
    }
    __syncthreads();
    {
        cd vv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int idx = el + 64 * j;
            const int row = idx / CHI, q = idx % CHI;
            const int iv = row / CHI, qb = row % CHI;
            cd acc = cz<double>();
#pragma unroll
            for (int iu = 0; iu < 2; ++iu) {
                cd part = cz<double>();
                for (int kk = 0; kk < CHI; ++kk) {
                    const double* b = Rv[iv] + 2 * (qb * CHI + kk);
                    part = ccfma(part, cd{b[0], b[1]}, Vl[iu * CHI + kk][q]);
                }
                acc = ccfma(acc, phl[iu][iv], part);
            }
            vv[j] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int idx = el + 64 * j;
            Vl[idx / CHI][idx % CHI] = vv[j];
        }
    }
    __syncthreads();
    for (int q = 0; q < CHI; ++q) {
        for (int pass = 0; pass < 2; ++pass) {
            cd upd = cz<double>();
            if (el < N) {
                for (int i = 0; i < q; ++i) {
                    cd dot = cz<double>();
                    for (int rr = 0; rr < N; ++rr) dot = ccfma(dot, Vl[rr][i], Vl[rr][q]);
                    upd = cfma(upd, dot, Vl[el][i]);
                }
            }
            __syncthreads();
            if (el < N) Vl[el][q] = csub(Vl[el][q], upd);
            __syncthreads();
        }
        double nq = 0.0;
        for (int rr = 0; rr < N; ++rr) nq += cabs2(Vl[rr][q]);
        const double inq = nq > 0.0 ? 1.0 / sqrt(nq) : 0.0;
        __syncthreads();
        if (el < N) Vl[el][q] = cscale(Vl[el][q], inq);
        __syncthreads();
    }
    // kept vectors per block: Z_b[row][q]
    for (int idx = el; idx < 4 * CHI * CHI; idx += 64) {
        const int b = idx / (CHI * CHI), row = (idx / CHI) % CHI, q = idx % CHI;
        const int crow = (b & 1) * CHI + row;
        const cd z = b < 2 ? Ul[crow][q] : cconj(Vl[crow][q]);
        double* dst = SuWs<CHI>::z(p.su_ws, ci, b) + 2 * (row * CHI + q);
        dst[0] = z.re;
        dst[1] = z.im;
    }
}

// Gamma_new (block b) = Q_b [Z_b; 0] divided by the outer lambdas
// (pseudo-inverse), QH output columns per pass (the reflectors are re-read
// per pass), reflectors applied last to first.
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k16_su_apply(DevPool p, const int32_t* items, int nc) {
    static_assert(CHI == 16, "chi = 16 layout");
    constexpr int ROWS = CHI * CHI;
    constexpr int RPL = ROWS / 64;
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int QH = 8;
    __shared__ double lamv[3][CHI];
    __shared__ double v2l[CHI];
    __shared__ cd Zl[CHI][CHI];
    const int b = blockIdx.x & 3, ci = blockIdx.x >> 2;
    if (ci >= nc) return;
    const int e = items[ci];
    const int lane = threadIdx.x;
    const int ib = b & 1;
    int vert, pleg, o1, o2;
    su_block_geometry<CHI>(p, e, b, vert, pleg, o1, o2);
    if (lane < 3 * CHI) lamv[lane / CHI][lane % CHI] = leg_lambda(p, vert, lane / CHI, lane % CHI, CHI);
    if (lane < CHI) v2l[lane] = SuWs<CHI>::v(p.su_ws, ci, b)[lane];
    {
        const double* zs = SuWs<CHI>::z(p.su_ws, ci, b);
        for (int idx = lane; idx < CHI * CHI; idx += 64) Zl[idx / CHI][idx % CHI] = {zs[2 * idx], zs[2 * idx + 1]};
    }
    __syncthreads();
    const int s1 = leg_stride<CHI>(o1), s2 = leg_stride<CHI>(o2), sp = leg_stride<CHI>(pleg);
    const double* H = SuWs<CHI>::h(p.su_ws, ci, b);
    cpx<S>* gdst = reinterpret_cast<cpx<S>*>(p.gam) + (size_t)vert * 2 * C3 + (size_t)ib * C3;
    double inv[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int row = lane + 64 * k;
        const double lo = lamv[o1][row / CHI] * lamv[o2][row % CHI];
        inv[k] = lo > 0.0 ? 1.0 / lo : 0.0;
    }
    // the column loop is not unrolled, so the QH columns' registers are
    // reused between passes
    for (int q0 = 0; q0 < CHI; q0 += QH) {
        cd z[QH][RPL];
#pragma unroll
        for (int qq = 0; qq < QH; ++qq)
#pragma unroll
            for (int k = 0; k < RPL; ++k) z[qq][k] = (k == 0 && lane < CHI) ? Zl[lane][q0 + qq] : cz<double>();
#pragma unroll
        for (int kc = CHI - 1; kc >= 0; --kc) {
            // reflector kc: rows >= kc of column kc
            cd hv[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int row = lane + 64 * k;
                const double* src = H + ((size_t)kc * ROWS + row) * 2;
                hv[k] = (k > 0 || lane >= kc) ? cd{src[0], src[1]} : cz<double>();
            }
            const double v2 = v2l[kc];
            double wsum[2 * QH];
#pragma unroll
            for (int qq = 0; qq < QH; ++qq) {
                cd w = cz<double>();
#pragma unroll
                for (int k = 0; k < RPL; ++k) w = ccfma(w, hv[k], z[qq][k]);
                wsum[2 * qq] = w.re;
                wsum[2 * qq + 1] = w.im;
            }
            wave_allreduce<2 * QH>(wsum, lane);
#pragma unroll
            for (int qq = 0; qq < QH; ++qq) {
                const cd f = cscale(cd{wsum[2 * qq], wsum[2 * qq + 1]}, v2);
#pragma unroll
                for (int k = 0; k < RPL; ++k) z[qq][k] = csub(z[qq][k], cmul(f, hv[k]));
            }
        }
#pragma unroll
        for (int qq = 0; qq < QH; ++qq)
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int row = lane + 64 * k;
                gdst[(row / CHI) * s1 + (row % CHI) * s2 + (q0 + qq) * sp] = from_cd<S>(cscale(z[qq][k], inv[k]));
            }
    }
}

// ------------------------------------------------------------------ Alg. 2 (chi = 16)
// One wavefront per edge; lane t owns the matrix elements u = t + 64 q
// (row u / chi, column u % chi).  Cholesky factors m = L L^dagger of the two
// messages (pivots <= eig_cut * max diag dropped), their pseudo-inverses by
// forward substitution (one column per lane), the bond core
// C[k][l] = sum_j L1[j][k] L2[j][l], its SVD by the team Jacobi, and the gauge
// maps X_u[j][q] = sqrt(lambda_old[j]) sum_j' Li1[j'][j] U[j'][q] (conj(V) for v).
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k16_canonicalise(DevPool p, const int32_t* items, int nitems) {
    if (tail_gated_off(p)) return;       // uniform: BP has not stopped
    static_assert(CHI == 16, "chi = 16 layout");
    constexpr int M2 = CHI * CHI;
    constexpr int EPT = M2 / 64;
    __shared__ cd A[2][CHI][CHI];
    __shared__ cd Li[2][CHI][CHI];
    __shared__ double sg[CHI];
    __shared__ int ordr[CHI];
    __shared__ double lold[CHI];
    __shared__ double diagmax[2];
    const int item = wg_index(p.xcd_remap);
    if (item >= nitems) return;
    const int e = items[item];
    const int t = threadIdx.x;
    const int slot = p.eslot[e];
    if (!(p.sflag[slot] & FLAG_ACTIVE)) return;     // uniform
    const cpx<S>* msg = reinterpret_cast<const cpx<S>*>(p.msg) + (size_t)e * 2 * M2;
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int u = t + 64 * q;
            A[w][u / CHI][u % CHI] = to_cd(msg[w * M2 + u]);
        }
    if (t < CHI) lold[t] = p.lam[(size_t)e * CHI + t];
    __syncthreads();
    if (t < 2) {
        double mx = 0.0;
        for (int j = 0; j < CHI; ++j) mx = fmax(mx, A[t][j][j].re);
        diagmax[t] = mx;
    }
    __syncthreads();
    for (int k = 0; k < CHI; ++k) {
        double dk[2];
#pragma unroll
        for (int w = 0; w < 2; ++w) dk[w] = A[w][k][k].re;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const bool piv = dk[w] > p.eig_cut * diagmax[w];
            const double s = piv ? sqrt(dk[w]) : 0.0;
            if (t >= k && t < CHI) A[w][t][k] = piv ? cscale(A[w][t][k], 1.0 / s) : cz<double>();
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < 2; ++w)
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const int u = t + 64 * q, r = u / CHI, c = u % CHI;
                if (r > k && c > k && c <= r) A[w][r][c] = csub(A[w][r][c], cmulc(A[w][r][k], A[w][c][k]));
            }
        __syncthreads();
    }
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int u = t + 64 * q, r = u / CHI, c = u % CHI;
            if (c > r) A[w][r][c] = cz<double>();
        }
    __syncthreads();
    if (t < 2 * CHI) {
        const int w = t / CHI, col = t % CHI;
        const double dcol = A[w][col][col].re;
        const bool live = dcol != 0.0;
        cd li[CHI];
#pragma unroll
        for (int i = 0; i < CHI; ++i) {
            const double di = A[w][i][i].re;
            const double rd = di != 0.0 ? 1.0 / di : 0.0;
            cd acc = cz<double>();
#pragma unroll
            for (int k = 0; k < i; ++k)
                if (k >= col) acc = cfma(acc, A[w][i][k], li[k]);
            li[i] = !live || i < col || rd == 0.0 ? cz<double>() : (i == col ? cd{rd, 0.0} : cscale(acc, -rd));
        }
#pragma unroll
        for (int i = 0; i < CHI; ++i) Li[w][i][col] = li[i];
    }
    __syncthreads();
    constexpr int LPC = JLayout<CHI, 64>::LPC;
    constexpr int EPL = JLayout<CHI, 64>::EPL;
    const int jcol = JLayout<CHI, 64>::col(t), jg = JLayout<CHI, 64>::grp(t);
    cd m[EPL], v[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int row = jg + LPC * k;
        cd acc = cz<double>();
        for (int j = 0; j < CHI; ++j) acc = cfma(acc, A[0][j][row], A[1][j][jcol]);
        m[k] = acc;
        v[k] = (row == jcol) ? cd{1.0, 0.0} : cz<double>();
    }
    const int sweeps = jacobi_svd_team<CHI, 64>(m, v, t, JACOBI_TOL, JACOBI_MAX_SWEEPS);
    if (sweeps > JACOBI_MAX_SWEEPS && t == 0) atomicOr(&p.swarn[slot], (int)WARN_JACOBI);
    double nl = 0.0;
#pragma unroll
    for (int k = 0; k < EPL; ++k) nl += cabs2(m[k]);
    nl = strided_sum<CHI, LPC>(nl);
    const double sgm = sqrt(nl);
    if (jg == 0) sg[jcol] = sgm;
    if (t < CHI) ordr[t] = t;
    __syncthreads();
    if (t < CHI) {
        int rank = 0;
        const double me = sg[t];
        for (int k = 0; k < CHI; ++k) {
            const double o = sg[k];
            rank += (o > me || (o == me && k < t)) ? 1 : 0;
        }
        if (rank < CHI) ordr[rank] = t;
    }
    __syncthreads();
    const double smax = sg[ordr[0]];
    int rk = 0;
    double kept2 = 0.0;
    for (int k = 0; k < CHI; ++k) {
        const double sk = sg[ordr[k]];
        if (sk > p.svd_cut * smax) {
            rk = k + 1;
            kept2 += sk * sk;
        }
    }
    {
        int dstq = 0;
        for (int k = 0; k < CHI; ++k)
            if (ordr[k] == jcol) dstq = k;
        const double isg = sgm > 0.0 ? 1.0 / sgm : 0.0;
        const bool keep = dstq < rk;
        __syncthreads();                     // every lane has read the factors for the core
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int row = jg + LPC * k;
            A[0][row][dstq] = keep ? cscale(m[k], isg) : cz<double>();
            A[1][row][dstq] = keep ? cconj(v[k]) : cz<double>();
        }
    }
    __syncthreads();
    cpx<S>* xg = reinterpret_cast<cpx<S>*>(p.xg) + (size_t)e * 2 * M2;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int u = t + 64 * q, r = u / CHI, c = u % CHI;
        const double sl = sqrt(lold[r]);
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            cd acc = cz<double>();
            for (int jp = 0; jp < CHI; ++jp) acc = cfma(acc, Li[w][jp][r], A[w][jp][c]);
            xg[w * M2 + u] = from_cd<S>(cscale(acc, sl));
        }
    }
    if (t < CHI) {
        const double inv = kept2 > 0.0 ? 1.0 / sqrt(kept2) : 0.0;
        p.lam[(size_t)e * CHI + t] = t < rk ? sg[ordr[t]] * inv : 0.0;
    }
}

// ------------------------------------------------------------------ Vidal residual
// The local-orthogonality residual of vertex a (App. C): for each leg b the
// Gram matrix M[j][j'] = sum over the other indices of Gamma_a[.., j]
// conj(Gamma_a[.., j']) times the squared lambdas of a's other legs, and the
// trace norm of D = delta_d - (d / tr M) M, d the bond dimension of b (M is
// compared with the identity after division by its mean eigenvalue, since
// Alg. 2 fixes Gamma_a only up to a positive scale).  One work-group of 256
// lanes per vertex, the tensor staged in LDS in its storage precision.  The
// Gram matrices: 30 groups of 8 lanes, a group per (leg, 4 x 4 block of the
// upper triangle), each lane summing one eighth of the 512 fibres (stride 8)
// in FP64, the eight partial blocks summed by xor shuffles.  The trace norm
// is the sum of D's singular values, by the 64-lane team Jacobi, one
// wavefront per leg.  The value is exact in every mode; RES_BOUNDS writes it
// as both bounds.
template <int CHI, typename S>
__global__ __launch_bounds__(256) void k16_residual(DevPool p, const int32_t* items, int nitems, int mode) {
    static_assert(CHI == 16, "chi = 16 layout");
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int NF = 2 * CHI * CHI;                // fibres per leg
    constexpr int PARTS = 8;
    __shared__ cpx<S> G[2 * C3];
    __shared__ double lam2[3][CHI];
    __shared__ int dims[3];
    __shared__ cd Mm[3][CHI][CHI];
    __shared__ double term[3];
    const int item = wg_index(p.xcd_remap);
    if (item >= nitems) return;                      // uniform
    const int a = items[item];
    if (mode == RES_UNDECIDED && !(p.sflag[p.vslot[a]] & FLAG_UNDECIDED)) return;   // uniform
    const int t = threadIdx.x;
    const cpx<S>* gam = reinterpret_cast<const cpx<S>*>(p.gam) + (size_t)a * 2 * C3;
    for (int idx = t; idx < 2 * C3; idx += 256) G[idx] = gam[idx];
    if (t < 3 * CHI) {
        const double lv = leg_lambda(p, a, t / CHI, t % CHI, CHI);
        lam2[t / CHI][t % CHI] = lv * lv;
    }
    if (t < 3) {
        const int e2 = p.vedge[3 * a + t];
        int dim = 0;
        if (e2 >= 0)
            for (int j = 0; j < CHI; ++j)
                if (p.lam[(size_t)e2 * CHI + j] > 0.0) dim = j + 1;
        dims[t] = dim;
    }
    __syncthreads();
    {
        // groups 30 and 31 (the last 16 lanes) repeat group 29 and store nothing
        const int grp = (t >> 3) < 30 ? (t >> 3) : 29;
        const int part = t & (PARTS - 1);
        const int lg = grp / 10;
        int blk = grp % 10, bj = 0;
        while (blk >= 4 - bj) {
            blk -= 4 - bj;
            ++bj;
        }
        const int bjp = bj + blk;                    // 4 x 4 block (bj, bjp), bj <= bjp
        int o1, o2;
        other_legs(lg, o1, o2);
        const int sb = leg_stride<CHI>(lg), s1 = leg_stride<CHI>(o1), s2 = leg_stride<CHI>(o2);
        cd acc[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = cz<double>();
        for (int f = part; f < NF; f += PARTS) {
            const int i = f / (CHI * CHI), k1 = (f / CHI) % CHI, k2 = f % CHI;
            const double w = lam2[o1][k1] * lam2[o2][k2];
            const int base = i * C3 + k1 * s1 + k2 * s2;
            cd x[4], y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                x[r] = cscale(to_cd(G[base + (4 * bj + r) * sb]), w);
                y[r] = to_cd(G[base + (4 * bjp + r) * sb]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = cfmac(acc[r][c], x[r], y[c]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                cd v = acc[r][c];
                v = cadd(v, shfl_xor_cd(v, 4));
                v = cadd(v, shfl_xor_cd(v, 2));
                v = cadd(v, shfl_xor_cd(v, 1));
                acc[r][c] = v;
            }
        if (part == 0 && (t >> 3) < 30) {
            const int dim = dims[lg];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int j = 4 * bj + r, jp = 4 * bjp + c;
                    const bool in = j < dim && jp < dim;
                    if (bj == bjp) {
                        // diagonal block: the Hermitian part of both halves
                        const cd h = cscale(cadd(acc[r][c], cconj(acc[c][r])), 0.5);
                        Mm[lg][j][jp] = in ? h : cz<double>();
                    } else {
                        Mm[lg][j][jp] = in ? acc[r][c] : cz<double>();
                        Mm[lg][jp][j] = in ? cconj(acc[r][c]) : cz<double>();
                    }
                }
        }
    }
    __syncthreads();
    const int wv = t >> 6, tl = t & 63;
    if (wv < 3) {                                    // one wavefront per leg
        constexpr int LPC = JLayout<CHI, 64>::LPC;
        constexpr int EPL = JLayout<CHI, 64>::EPL;
        const int jcol = JLayout<CHI, 64>::col(tl), jg = JLayout<CHI, 64>::grp(tl);
        const int dim = dims[wv];
        double tr = 0.0;
        for (int q = 0; q < CHI; ++q) tr += Mm[wv][q][q].re;
        const double sc = tr > 0.0 ? dim / tr : 0.0;
        cd m[EPL], vdummy[EPL];
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int row = jg + LPC * k;
            cd dv = cscale(Mm[wv][row][jcol], -sc);
            if (row == jcol && row < dim) dv.re += 1.0;
            m[k] = dv;
        }
        jacobi_svd_team<CHI, 64, false>(m, vdummy, tl, JACOBI_TOL, JACOBI_MAX_SWEEPS);
        double nrm = 0.0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) nrm += cabs2(m[k]);
        nrm = strided_sum<CHI, LPC>(nrm);
        double sv = jg == 0 ? sqrt(nrm) : 0.0;
        sv = seg_sum<64>(sv);
        if (tl == 0) term[wv] = dim > 0 ? sv : 0.0;
    }
    __syncthreads();
    if (t == 0) {
        const double r = term[0] + term[1] + term[2];
        p.vres[a] = r;
        if (mode == RES_BOUNDS) p.vres_hi[a] = r;
    }
}

// ------------------------------------------------------------------ launchers
static int wide_err() { return hipGetLastError() == hipSuccess ? 0 : -4; }

#define GTQA_WIDE_DISPATCH(chi, prec, CALL)                                       \
    do {                                                                           \
        if ((chi) == 16 && (prec) == 0) { constexpr int CHI = 16; using S = double; CALL; } \
        else if ((chi) == 16) { constexpr int CHI = 16; using S = float; CALL; }    \
        else return -1;                                                            \
    } while (0)

static unsigned wide_grid(DevPool& q, long groups) {
    q.xcd_remap = tuning().xcd_remap;
    if (q.xcd_remap) groups = (groups + 7) / 8 * 8;
    return (unsigned)groups;
}

int launch_wide_simple_update(int chi, int prec, const DevPool& p, const int32_t* edges, int ne, hipStream_t s) {
    if (ne <= 0) return 0;
    if (!p.su_ws || p.su_chunk <= 0) return -1;
    GTQA_WIDE_DISPATCH(chi, prec, ({
        for (int off = 0; off < ne; off += p.su_chunk) {
            const int nc = ne - off < p.su_chunk ? ne - off : p.su_chunk;
            k16_su_qr<CHI, S><<<4 * nc, 64, 0, s>>>(p, edges + off, nc);
            k16_su_core<CHI, S><<<nc, 64, 0, s>>>(p, edges + off, nc);
            k16_su_apply<CHI, S><<<4 * nc, 64, 0, s>>>(p, edges + off, nc);
        }
    }));
    return wide_err();
}

int launch_wide_bp_sweep_class(int chi, int prec, const DevPool& p, const int4* recs, int ne, int first_sweep,
                               int cls, const int32_t* gate, hipStream_t s) {
    if (ne <= 0) return 0;
    DevPool q = p;
    GTQA_WIDE_DISPATCH(chi, prec, ({
        const unsigned grid = wide_grid(q, ne);
        // the first sweep's first class (every class of a flooding first
        // sweep) sees only diagonal incoming messages
        if (p.bp_flood) {
            if (first_sweep) k16_bp_class<CHI, S, true, true, true><<<grid, 256, 0, s>>>(q, recs, ne, cls, gate);
            else k16_bp_class<CHI, S, false, true><<<grid, 256, 0, s>>>(q, recs, ne, cls, gate);
        } else {
            if (first_sweep && cls == 0)
                k16_bp_class<CHI, S, true, false, true><<<grid, 256, 0, s>>>(q, recs, ne, cls, gate);
            else if (first_sweep) k16_bp_class<CHI, S, true, false><<<grid, 256, 0, s>>>(q, recs, ne, cls, gate);
            else k16_bp_class<CHI, S, false, false><<<grid, 256, 0, s>>>(q, recs, ne, cls, gate);
        }
    }));
    return wide_err();
}

int launch_wide_residual(int chi, int prec, const DevPool& p, const int32_t* verts, int nv, int mode,
                         hipStream_t s) {
    if (nv <= 0) return 0;
    DevPool q = p;
    GTQA_WIDE_DISPATCH(chi, prec, (k16_residual<CHI, S><<<wide_grid(q, nv), 256, 0, s>>>(q, verts, nv, mode)));
    return wide_err();
}

int launch_wide_canonicalise(int chi, int prec, const DevPool& p, const int32_t* edges, int ne, hipStream_t s) {
    if (ne <= 0) return 0;
    DevPool q = p;
    GTQA_WIDE_DISPATCH(chi, prec, (k16_canonicalise<CHI, S><<<wide_grid(q, ne), 64, 0, s>>>(q, edges, ne)));
    return wide_err();
}

int launch_wide_gauge_apply(int chi, int prec, const DevPool& p, const int32_t* verts, int nv, int apply_x,
                            hipStream_t s) {
    if (nv <= 0) return 0;
    DevPool q = p;
    GTQA_WIDE_DISPATCH(chi, prec, (k16_gauge_apply<CHI, S><<<wide_grid(q, nv), 128, 0, s>>>(q, verts, nv, apply_x)));
    return wide_err();
}

}  // namespace gtqa
