// HIP kernels (gfx950) of the GTQA Trotter step.
//
// Every kernel runs one 64-lane wavefront per workgroup.  Work items (edges
// or vertices of possibly many instances) are taken from index lists; a
// "team" of lanes owns one item and keeps small dense matrices in
// registers, exchanging values with cross-lane shuffles and LDS.
//
//   k_simple_update   two-qubit gate on one edge (App. E) + truncation
//                     (Alg. 3): QR of the four physical blocks of the two
//                     site tensors, 2chi x 2chi core, one-sided Jacobi SVD,
//                     new Gamma_u, Gamma_v, lambda_e.  FP64 throughout.
//   k_warm_messages   BP start messages diag(lambda)/sum(lambda) (Sec. II.C).
//   k_bp_class        one colour class of an in-place BP sweep (Alg. 1):
//                     both messages of each edge, unit trace, trace-norm
//                     distance.
//   k_bp_reduce       per-instance distance sum in a fixed order and the
//                     stop decision.
//   k_canonicalise    Alg. 2 per edge in FP64: factor the two messages,
//                     SVD of the bond core, gauge maps, new lambda.
//   k_gauge_apply     Gamma_a <- T_a contracted with the gauge maps of its
//                     three legs; optionally followed by exp(-i theta X).
//   k_x_layer, k_readout, k_energy, k_init_plus: the rest of the step.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>

#include "gtqa.h"
#include "gtqa_internal.h"
#include "gtqa_device.h"

namespace gtqa {

// ------------------------------------------------------------------ init
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_init_plus(DevPool p, const int32_t* verts, int nv,
                                                  const int32_t* edges, int ne) {
    constexpr int G = 2 * CHI * CHI * CHI;
    cpx<S>* gam = reinterpret_cast<cpx<S>*>(p.gam);
    const size_t gid = (size_t)blockIdx.x * 64 + threadIdx.x;
    const size_t totv = (size_t)nv * G;
    if (gid < totv) {
        const int a = verts[gid / G];
        const int idx = (int)(gid % G);
        const S val = (idx % (CHI * CHI * CHI) == 0) ? S(0.70710678118654752440) : S(0);
        gam[(size_t)a * G + idx] = {val, S(0)};
    }
    const size_t tote = (size_t)ne * CHI;
    if (gid < tote) {
        const int e = edges[gid / CHI];
        const int j = (int)(gid % CHI);
        p.lam[(size_t)e * CHI + j] = (j == 0) ? 1.0 : 0.0;
    }
}

// ------------------------------------------------------------------ simple update
// EPW edges per workgroup (one wavefront), LPE = 64/EPW lanes per edge.
// Within an edge, lanes [b*LPB, (b+1)*LPB) own block b of the four physical
// blocks: b = 0,1 -> Gamma_u[i = b] scaled by the outer lambdas of u and by
// lambda_e on the bond leg; b = 2,3 -> Gamma_v[i = b-2] scaled by the outer
// lambdas of v.  Each block is a chi^2 x chi matrix (rows: the two outer
// legs, columns: the bond leg); a lane holds RPL of its rows.
// The register budget is capped at three wavefronts per SIMD at chi <= 4 and
// two at chi = 8: the Jacobi phase is latency bound and gains more from the
// extra wavefront than the values held in scratch across it cost (measured:
// chi = 8 one wavefront 3.2 ms, two 2.1 ms, three 2.9 ms per launch of
// 24,000 edges).
// FIX = false: the bond SVD rotates only pairs touching the CHI largest core
// columns (at CHI <= 4) and then checks kept_set_is_largest; an edge that
// fails the check (or does not settle in KEEP_SWEEPS sweeps) writes nothing
// but its flag in p.efix.  FIX = true, launched right after over the same
// list: only flagged edges run, with the plain every-pair Jacobi; a
// work-group without a flagged edge returns at once.  Keeping the rare
// fallback in its own instantiation leaves the common kernel's register
// footprint that of the restricted iteration alone.
template <int CHI, typename S, int EPW, bool FIX = false>
__global__ __launch_bounds__(64, CHI <= 4 ? 3 : 2) void k_simple_update(DevPool p, const int32_t* items, int nitems) {
    constexpr int LPE = 64 / EPW;            // lanes per edge
    constexpr int LPB = LPE / 4;             // lanes per physical block
    constexpr int R = CHI * CHI;
    constexpr int RPL = R / LPB;             // block rows per lane
    constexpr int N = 2 * CHI;
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int LPC = JLayout<N, LPE>::LPC;
    constexpr int EPL = JLayout<N, LPE>::EPL;
    static_assert(R % LPB == 0 && RPL >= 1, "block rows must divide over the lanes");
    static_assert(LPB >= CHI, "the R factor rows must sit in distinct lanes");

    __shared__ double lamv[EPW][2][3][CHI];
    __shared__ cd Rl[EPW][4][CHI][CHI];
    __shared__ double v2l[EPW][4][CHI];     // 2/|v|^2 of the Householder reflectors
    // the core before the SVD: kept in LDS for chi > 4; for chi <= 4 the
    // rows needed later are recomputed from the R factors and gate phases
    __shared__ cd Tl[CHI <= 4 ? 1 : EPW][N][N];
    __shared__ cd phl[EPW][2][2];            // gate phases phi(iu, iv)
    __shared__ cd Ul[EPW][N][N];
    __shared__ cd Vl[EPW][N][CHI];           // kept right singular vectors, by rank
    __shared__ double sig[EPW][N];
    __shared__ int order[EPW][N];

    const int lane = threadIdx.x;
    const int sub = lane / LPE;              // edge within the workgroup
    const int el = lane % LPE;               // lane within the edge
    const int item = wg_index(p.xcd_remap) * EPW + sub;
    bool valid = item < nitems;              // padding lanes recompute items[0], write nothing
    const int e = items[valid ? item : 0];
    if constexpr (FIX) {
        valid = valid && p.efix[e] != 0;
        if (__ballot(valid) == 0) return;    // uniform over the work-group (one wavefront)
    }
    const int slot = p.eslot[e];
    const int b = el / LPB;
    const int l = el % LPB;
    const int side = b >> 1;
    const int ib = b & 1;
    const int uv[2] = {p.eend[2 * e], p.eend[2 * e + 1]};
    const int pl[2] = {p.eleg[2 * e], p.eleg[2 * e + 1]};
    const double theta = p.theta[2 * slot];

    // lambdas of both endpoints' legs, addressed from the BP direction records
    for (int idx = el; idx < 2 * 3 * CHI; idx += LPE) {
        const int sd = idx / (3 * CHI), lg = (idx / CHI) % 3, j = idx % CHI;
        const int4 md = p.bpmeta[2 * e + sd];
        const int pleg = md.w & 3;
        int o1, o2;
        other_legs(pleg, o1, o2);
        const int inc = lg == pleg ? 2 * e : (lg == o1 ? md.y : md.z);
        lamv[sub][sd][lg][j] = inc >= 0 ? p.lam[(size_t)(inc >> 1) * CHI + j] : (j == 0 ? 1.0 : 0.0);
    }
    __syncthreads();

    // ---- load the block into registers: xr[k][j], row = l + LPB k
    const int vert = uv[side];
    const int pleg = pl[side];
    int o1, o2;
    other_legs(pleg, o1, o2);
    const int s1 = leg_stride<CHI>(o1), s2 = leg_stride<CHI>(o2), sp = leg_stride<CHI>(pleg);
    const cpx<S>* gsrc = reinterpret_cast<const cpx<S>*>(p.gam) + (size_t)vert * 2 * C3 + ib * C3;
    cd xr[RPL][CHI];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int row = l + LPB * k;
        const int j1 = row / CHI, j2 = row % CHI;
        const double sc = lamv[sub][side][o1][j1] * lamv[sub][side][o2][j2];
#pragma unroll
        for (int j = 0; j < CHI; ++j) {
            const double sj = side == 0 ? sc * lamv[sub][0][pl[0]][j] : sc;
            xr[k][j] = cscale(to_cd(gsrc[j1 * s1 + j2 * s2 + j * sp]), sj);
        }
    }

    // ---- Householder QR of the block (LPB lanes).  Reflector kc is
    // v = (top, x[kc+1:, kc]), kept in place (top in row kc, i.e. in lane kc
    // of the block since LPB >= CHI), with v2l[kc] = 2/|v|^2 (0: no
    // reflection).  The diagonal of R, which row kc held, goes to rdiag.
    cd rdiag = cz<double>();
    double v2inv[CHI];
#pragma unroll
    for (int kc = 0; kc < CHI; ++kc) {
        double part = 0.0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int row = l + LPB * k;
            if (row >= kc) part += cabs2(xr[k][kc]);
        }
        const double nrm2 = seg_sum<LPB>(part);
        // alpha = x[kc][kc], owned by lane kc % LPB of the block, slot kc / LPB
        cd alpha;
        if constexpr (LPB == 4) {
            const cd own = xr[kc / LPB][kc];
            alpha = {quad_bcast(own.re, kc % LPB), quad_bcast(own.im, kc % LPB)};
        } else {
            alpha = shfl_cd<LPB>(xr[kc / LPB][kc], kc % LPB);
        }
        const double nrm = sqrt(nrm2);
        const double aa = sqrt(cabs2(alpha));
        if (nrm > 0.0) {
            const cd ph = aa > 0.0 ? cd{alpha.re / aa, alpha.im / aa} : cd{1.0, 0.0};
            const cd top = {alpha.re + ph.re * nrm, alpha.im + ph.im * nrm};
            const double vv = 2.0 * nrm * (nrm + aa);
            v2inv[kc] = 2.0 / vv;
#pragma unroll
            for (int jc = kc + 1; jc < CHI; ++jc) {
                cd w = cz<double>();
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int row = l + LPB * k;
                    if (row > kc) w = ccfma(w, xr[k][kc], xr[k][jc]);
                    else if (row == kc) w = ccfma(w, top, xr[k][jc]);
                }
                w = seg_sum<LPB>(w);
                const cd f = cscale(w, v2inv[kc]);
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int row = l + LPB * k;
                    if (row > kc) xr[k][jc] = csub(xr[k][jc], cmul(f, xr[k][kc]));
                    else if (row == kc) xr[k][jc] = csub(xr[k][jc], cmul(f, top));
                }
            }
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                if (l + LPB * k == kc) {
                    rdiag = {-ph.re * nrm, -ph.im * nrm};
                    xr[k][kc] = top;
                }
            }
        } else {
            v2inv[kc] = 0.0;
        }
    }
    // R (upper triangle of the first CHI rows: lanes l < CHI, slot 0) and the
    // reflector scales to LDS
    if (l < CHI) {
#pragma unroll
        for (int j = 0; j < CHI; ++j) Rl[sub][b][l][j] = j > l ? xr[0][j] : (j == l ? rdiag : cz<double>());
    }
    if (l == 0) {
#pragma unroll
        for (int kc = 0; kc < CHI; ++kc) v2l[sub][b][kc] = v2inv[kc];
    }
    __syncthreads();

    // ---- core M[(iu,pa),(iv,qb)] = phi(iu,iv) sum_k R_A,iu[pa][k] R_B,iv[qb][k]
    const int ccol = JLayout<N, LPE>::col(el);
    const int cg = JLayout<N, LPE>::grp(el);
    const double Je = p.J[e];
    const double hu = p.hD[uv[0]], hv = p.hD[uv[1]];
    cd m[EPL], v[EPL];
    // the four gate phases phi(iu, iv), one per lane of the edge's first
    // four (an FP64 sincos is costly), then this lane's column's two
    cd ph[2];
    if (el < 4) {
        const int iu = el >> 1, iv = el & 1;
        const double zu = iu ? -1.0 : 1.0, zv = iv ? -1.0 : 1.0;
        const double ang = -theta * (Je * zu * zv + hu * zu + hv * zv);
        double sn, cs;
        sincos(ang, &sn, &cs);
        phl[sub][iu][iv] = {cs, sn};
    }
    __syncthreads();
    ph[0] = phl[sub][0][ccol / CHI];
    ph[1] = phl[sub][1][ccol / CHI];
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int row = cg + LPC * k;
        const int iu = row / CHI, pa = row % CHI;
        const int iv = ccol / CHI, qb = ccol % CHI;
        cd acc = cz<double>();
#pragma unroll
        for (int kk = 0; kk < CHI; ++kk) acc = cfma(acc, Rl[sub][iu][pa][kk], Rl[sub][2 + iv][qb][kk]);
        m[k] = cmul(acc, iu ? ph[1] : ph[0]);
        if constexpr (CHI > 4) Tl[sub][row][ccol] = m[k];
    }
    // The columns enter the Jacobi sorted by norm (descending, ties by
    // index): on these cores that ordering needs about 5% fewer sweeps.  Only
    // the column order changes, so U and sigma are unaffected, and V is
    // recovered below from the core itself.
    {
        double own2 = 0.0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) own2 += cabs2(m[k]);
        own2 = strided_sum<N, LPC>(own2);
        if (cg == 0) sig[sub][ccol] = own2;
        __syncthreads();
        int rk = 0;
        const double me = sig[sub][ccol];
        for (int c = 0; c < N; ++c) {
            const double o = sig[sub][c];
            rk += (o > me || (o == me && c < ccol)) ? 1 : 0;
        }
#pragma unroll
        for (int k = 0; k < EPL; ++k) Ul[sub][cg + LPC * k][rk] = m[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < EPL; ++k) m[k] = Ul[sub][cg + LPC * k][ccol];
    }
    // One-sided Jacobi without accumulating V: the columns become U Sigma.
    // The kept right vectors are recovered below as Theta^dagger U / sigma.
    // (the kept-column restriction pays at chi = 4; at chi = 8 its ranking of
    // 16 columns costs more than the sweeps it saves: 2.07 vs 2.44 ms)
    constexpr int KEEP = (CHI <= 4 && !FIX) ? CHI : N;
    const int sweeps =
        jacobi_svd_team<N, LPE, false, KEEP>(m, v, el, JACOBI_TOL, KEEP < N ? KEEP_SWEEPS : JACOBI_MAX_SWEEPS);
    bool ok = true;
    if constexpr (KEEP < N) {
        ok = sweeps <= KEEP_SWEEPS && kept_set_is_largest<N, LPE, KEEP>(m, el, p.svd_cut);
        if (valid && el == 0) p.efix[e] = ok ? 0 : 1;
    }
    const bool wr = valid && ok;             // failed edges are redone by the FIX launch
    if (wr && sweeps > JACOBI_MAX_SWEEPS && el == 0) atomicOr(&p.swarn[slot], (int)WARN_JACOBI);

    double nrm_loc = 0.0;
#pragma unroll
    for (int k = 0; k < EPL; ++k) nrm_loc += cabs2(m[k]);
    nrm_loc = strided_sum<N, LPC>(nrm_loc);
    const double sgm = sqrt(nrm_loc);
    if (cg == 0) sig[sub][ccol] = sgm;
    if (el < N) order[sub][el] = el;   // stays a permutation even for NaN input
    __syncthreads();
    if (el < N) {
        int rank = 0;
        const double me = sig[sub][el];
        for (int c = 0; c < N; ++c) {
            const double o = sig[sub][c];
            rank += (o > me || (o == me && c < el)) ? 1 : 0;
        }
        if (rank < N) order[sub][rank] = el;
    }
    __syncthreads();
    const double smax = sig[sub][order[sub][0]];
    int r = 0;
    double kept2 = 0.0;
    for (int k = 0; k < CHI; ++k) {
        const double sk = sig[sub][order[sub][k]];
        if (sk > p.svd_cut * smax) {
            r = k + 1;
            kept2 += sk * sk;
        }
    }
    const double inv_norm = kept2 > 0.0 ? 1.0 / sqrt(kept2) : 0.0;
    if (wr && el == 0) {
        // gate fidelity estimate f = (sum_kept sigma^2 / sum sigma^2)^2 on the
        // normalised spectrum before truncation, and eps_ab^chi (Sec. II.C)
        double tot = 0.0, dropped = 0.0;
        for (int k = 0; k < N; ++k) {
            const double sk = sig[sub][order[sub][k]];
            tot += sk * sk;
            if (k >= r) dropped += sk * sk;
        }
        p.elogf[e] = tot > 0.0 ? 2.0 * log(kept2 / tot) : 0.0;
        p.eeps[e] = tot > 0.0 ? sqrt(dropped / tot) : 0.0;
    }
    // U = (Theta V) columns / sigma to LDS (columns in original order)
    {
        const double isg = sgm > 0.0 ? 1.0 / sgm : 0.0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int row = cg + LPC * k;
            Ul[sub][row][ccol] = cscale(m[k], isg);
        }
    }
    if (wr && el < CHI) {
        p.lam[(size_t)e * CHI + el] = el < r ? sig[sub][order[sub][el]] * inv_norm : 0.0;
    }
    __syncthreads();
    // kept right singular vectors by rank: w_q = Theta^dagger u_q / sigma_q
    // (exact in exact arithmetic), then re-orthonormalised by one Cholesky-QR
    // pass: the columns of w are unit vectors up to rounding that Theta^dagger
    // spreads into the directions of larger singular values (relative size
    // eps sigma_0 / sigma_q), so their Gram matrix is the identity to that
    // order and its Cholesky factor is well conditioned.  Lane el < N holds
    // row el; the other lanes hold zeros.  (The register form is used up to
    // chi = 4; larger chi runs two Gram-Schmidt passes in LDS.)
    if constexpr (CHI <= 4) {
        cd w[CHI];
        const int row = el < N ? el : 0;
        // column `row` of the core, recomputed exactly as it was formed
        cd mcol[N];
        {
            const int iv = row / CHI, qb = row % CHI;
#pragma unroll
            for (int pp = 0; pp < N; ++pp) {
                const int iu = pp / CHI, pa = pp % CHI;
                cd acc = cz<double>();
#pragma unroll
                for (int kk = 0; kk < CHI; ++kk) acc = cfma(acc, Rl[sub][iu][pa][kk], Rl[sub][2 + iv][qb][kk]);
                mcol[pp] = cmul(acc, phl[sub][iu][iv]);
            }
        }
#pragma unroll
        for (int q = 0; q < CHI; ++q) {
            cd acc = cz<double>();
            if (el < N && q < r) {
                const int src = order[sub][q];
                for (int pp = 0; pp < N; ++pp) acc = ccfma(acc, mcol[pp], Ul[sub][pp][src]);
                const double sq = sig[sub][src];
                acc = cscale(acc, 1.0 / sq);
            }
            w[q] = acc;
        }
        // Gram G[i][k] = sum_rows conj(w_i) w_k, upper triangle, summed over
        // lanes el < N, which hold the N rows (the other lanes' results are
        // not used)
        static_assert((N & (N - 1)) == 0 && N <= LPE, "rows must fill an aligned power-of-two lane group");
        cd Gm[CHI][CHI];
#pragma unroll
        for (int i = 0; i < CHI; ++i)
#pragma unroll
            for (int k = i; k < CHI; ++k) Gm[i][k] = seg_sum<N>(ccfma(cz<double>(), w[i], w[k]));
        // G = R^dagger R, R upper triangular; zero columns (q >= r) stay zero
        cd Rm[CHI][CHI];
        double rinv[CHI];
#pragma unroll
        for (int k = 0; k < CHI; ++k) {
            double dk = Gm[k][k].re;
#pragma unroll
            for (int i = 0; i < k; ++i) dk -= cabs2(Rm[i][k]);
            const bool piv = dk > 0.0 && k < r;
            rinv[k] = piv ? rsqrt(dk) : 0.0;
#pragma unroll
            for (int j = k + 1; j < CHI; ++j) {
                cd g = Gm[k][j];
#pragma unroll
                for (int i = 0; i < k; ++i) g = csub(g, ccfma(cz<double>(), Rm[i][k], Rm[i][j]));
                Rm[k][j] = cscale(g, rinv[k]);
            }
            Rm[k][k] = {piv ? dk * rinv[k] : 0.0, 0.0};
        }
        // x = w R^{-1}, row by row: x_k = (w_k - sum_{i<k} x_i R[i][k]) / R[k][k]
        cd x[CHI];
#pragma unroll
        for (int k = 0; k < CHI; ++k) {
            cd acc = w[k];
#pragma unroll
            for (int i = 0; i < k; ++i) acc = csub(acc, cmul(x[i], Rm[i][k]));
            x[k] = cscale(acc, rinv[k]);
        }
        if (el < N) {
#pragma unroll
            for (int q = 0; q < CHI; ++q) Vl[sub][el][q] = x[q];
        }
        __syncthreads();
    } else {
        for (int idx = el; idx < N * CHI; idx += LPE) {
            const int row = idx % N, q = idx / N;
            cd w = cz<double>();
            if (q < r) {
                const int src = order[sub][q];
                for (int pp = 0; pp < N; ++pp) w = ccfma(w, Tl[sub][pp][row], Ul[sub][pp][src]);
            }
            Vl[sub][row][q] = w;
        }
        __syncthreads();
        // uniform trip count: columns q >= r are zero and stay zero
        for (int q = 0; q < CHI; ++q) {
            for (int pass = 0; pass < 2; ++pass) {
                cd upd = cz<double>();
                if (el < N) {
                    for (int i = 0; i < q; ++i) {
                        cd dot = cz<double>();
                        for (int rr = 0; rr < N; ++rr) dot = ccfma(dot, Vl[sub][rr][i], Vl[sub][rr][q]);
                        upd = cfma(upd, dot, Vl[sub][el][i]);
                    }
                }
                __syncthreads();
                if (el < N) Vl[sub][el][q] = csub(Vl[sub][el][q], upd);
                __syncthreads();
            }
            double nq = 0.0;
            for (int rr = 0; rr < N; ++rr) nq += cabs2(Vl[sub][rr][q]);
            const double inq = nq > 0.0 ? 1.0 / sqrt(nq) : 0.0;
            __syncthreads();
            if (el < N) Vl[sub][el][q] = cscale(Vl[sub][el][q], inq);
            __syncthreads();
        }
    }
    // ---- Gamma_new = Q_block * [Z; 0], Z = U (side u) or conj(V) (side v),
    // one output column q at a time; then divided by the outer lambdas
    // (pseudo-inverse) and stored
    cpx<S>* gdst = reinterpret_cast<cpx<S>*>(p.gam) + (size_t)vert * 2 * C3 + ib * C3;
    double inv[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int row = l + LPB * k;
        const double lo = lamv[sub][side][o1][row / CHI] * lamv[sub][side][o2][row % CHI];
        inv[k] = lo > 0.0 ? 1.0 / lo : 0.0;
    }
#pragma unroll
    for (int q = 0; q < CHI; ++q) {
        cd z[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int row = l + LPB * k;
            z[k] = cz<double>();
            if (row < CHI && q < r) {
                const int crow = ib * CHI + row;
                z[k] = side == 0 ? Ul[sub][crow][order[sub][q]] : cconj(Vl[sub][crow][q]);
            }
        }
#pragma unroll
        for (int kc = CHI - 1; kc >= 0; --kc) {
            cd w = cz<double>();
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                if (l + LPB * k >= kc) w = ccfma(w, xr[k][kc], z[k]);
            }
            w = seg_sum<LPB>(w);
            const cd f = cscale(w, v2l[sub][b][kc]);
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                if (l + LPB * k >= kc) z[k] = csub(z[k], cmul(f, xr[k][kc]));
            }
        }
        if (wr) {
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int row = l + LPB * k;
                gdst[(row / CHI) * s1 + (row % CHI) * s2 + q * sp] = from_cd<S>(cscale(z[k], inv[k]));
            }
        }
    }
}

// ------------------------------------------------------------------ BP
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_warm_messages(DevPool p, const int32_t* items, int nitems) {
    const size_t gid = (size_t)blockIdx.x * 64 + threadIdx.x;
    constexpr int M2 = CHI * CHI;
    if (gid >= (size_t)nitems * 2 * M2) return;
    const int e = items[gid / (2 * M2)];
    if (!(p.sflag[p.eslot[e]] & FLAG_ACTIVE)) return;
    const int rem = (int)(gid % (2 * M2));
    const int idx = rem % M2;
    const int r = idx / CHI, c = idx % CHI;
    double tot = 0.0;
    for (int j = 0; j < CHI; ++j) tot += p.lam[(size_t)e * CHI + j];
    const double val = (r == c && tot > 0.0) ? p.lam[(size_t)e * CHI + r] / tot : 0.0;
    cpx<S>* msg = reinterpret_cast<cpx<S>*>(p.msg);
    msg[(size_t)e * 2 * M2 + rem] = {S(val), S(0)};
}

// Messages a -> b for both directions of EPG edges per group, DL lanes per
// direction (two edges and 16 lanes per direction at chi <= 4, one edge and
// 32 lanes at chi = 8).
// m_out[j, j'] = sum T[i, j@p, k@o1, l@o2] conj(T[i, j'@p, k'@o1, l'@o2]) m1[k, k'] m2[l, l']
// with T = Gamma_a * prod sqrt(lambda) (Eq. symmetric_gauge).  The distance
// of the stop test is bracketed: ||D||_F <= ||D||_1 <= min(sqrt(chi)||D||_F,
// sum |D_ij|); the replaced message is kept for the exact pass.
// The work record is the only load the others depend on: the tensor, lambda,
// message and flag loads are issued together right after it, unconditionally
// (addresses clamped to valid entries), and the warm-start messages are
// formed from the lambdas once they are in LDS.  (Running several groups per
// work-group with the next group's loads in flight during the current one's
// compute measured slower: the extra registers cost more resident wavefronts
// than the overlap gains.)
template <int CHI>
struct BPLayout {
    static constexpr int DPW = CHI <= 4 ? 4 : 2;   // directions per work-group
    static constexpr int DL = 64 / DPW;            // lanes per direction
    static constexpr int EPG = DPW / 2;            // edges per work-group
};

// Per-lane registers of one direction: its record and everything it loads
// (values a lane does not use, for missing legs or warm-start messages, are
// replaced when computing).
template <int CHI, typename S>
struct BPRegs {
    static constexpr int M2 = CHI * CHI;
    static constexpr int DL = BPLayout<CHI>::DL;
    static constexpr int MPL = M2 / DL;
    static constexpr int GPL = 2 * CHI * CHI * CHI / DL;
    static constexpr bool GREG = GPL <= 8;         // stage the tensor in registers
    int4 md;                                       // direction record
    int e, slot, fl;
    double lv;                                     // lambda of leg hl / CHI at index hl % CHI
    cpx<S> mreg[2][MPL];                           // incoming messages as stored
    cpx<S> oldr[MPL];                              // this direction's stored message
    cpx<S> greg[GREG ? GPL : 1];
};

template <int CHI>
__device__ __forceinline__ void bp_record(const int4* recs, int nitems, int g, int d, int4& md, int4& es) {
    constexpr int EPG = BPLayout<CHI>::EPG;
    int item = g * EPG + d / 2;
    if (item >= nitems) item = g * EPG;            // past the end: the work-group's first item
    const int4* rec = recs + 3 * (size_t)item;
    md = rec[d & 1];
    es = rec[2];
}

template <int CHI, typename S, bool FIRST, bool FLOOD>
__device__ __forceinline__ void bp_load(const DevPool& p, int4 md, int4 es, int d, int hl, int cls,
                                        BPRegs<CHI, S>& r) {
    using W = cpx<S>;
    constexpr int M2 = CHI * CHI;
    constexpr int DL = BPLayout<CHI>::DL;
    constexpr int MPL = BPRegs<CHI, S>::MPL;
    r.md = md;
    r.e = es.x;
    r.slot = es.y;
    const int pleg = md.w & 3;
    int o1, o2;
    other_legs(pleg, o1, o2);
    {
        const int h = hl < 3 * CHI ? hl : 3 * CHI - 1;
        const int lg = h / CHI, j = h % CHI;
        const int inc = lg == pleg ? 2 * es.x : (lg == o1 ? md.y : md.z);
        const double v = p.lam[(size_t)(inc >= 0 ? inc >> 1 : 0) * CHI + j];
        r.lv = inc >= 0 ? v : (j == 0 ? 1.0 : 0.0);
    }
    // flooding reads the previous iterate (mold), colour order the current one
    const W* msg = reinterpret_cast<const W*>(FLOOD ? p.mold : p.msg);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        // missing legs and warm-start messages read message 0 instead (a
        // cache hit shared by every such lane; the value is replaced)
        const int inc = w == 0 ? md.y : md.z;
        const int col = (md.w >> (8 + 8 * w)) & 255;
        const bool stored = inc >= 0 && !(FIRST && (FLOOD || col > cls));
        const W* in = msg + (size_t)(stored ? inc : 0) * M2;
#pragma unroll
        for (int k = 0; k < MPL; ++k) r.mreg[w][k] = in[hl + DL * k];
    }
    if (!FIRST) {
        const W* own = msg + ((size_t)es.x * 2 + (d & 1)) * M2;
#pragma unroll
        for (int k = 0; k < MPL; ++k) r.oldr[k] = own[hl + DL * k];
    }
    if (BPRegs<CHI, S>::GREG) {
        const W* gsrc = reinterpret_cast<const W*>(p.gam) + (size_t)md.x * 2 * CHI * CHI * CHI;
#pragma unroll
        for (int k = 0; k < BPRegs<CHI, S>::GPL; ++k) r.greg[k] = gsrc[hl + DL * k];
    }
    r.fl = p.sflag[es.y];
}

// gate (may be null): the count of slots still sweeping after the previous
// sweep's stop test; 0 means every slot has stopped and the launch returns
// at once (sweeps enqueued ahead of the host's read-back).
// FLOOD: flooding schedule, every incoming message from the previous
// iterate (in mold, snapshot before the sweep; the warm start in the first
// sweep), so the classes of a sweep do not depend on each other.
// WARM (with FIRST): every incoming message is diagonal, as in the first
// sweep's first class, whose neighbouring edges all belong to classes not yet
// visited (and in a flooding schedule's first sweep); the two mode products
// with the incoming messages are then scalings (the values the full products
// give: their off-diagonal terms add exact zeros); at chi = 4 the last
// contraction runs over the lane's own order of the third index, at chi = 8
// the two scalings share one pass through LDS.
template <int CHI, typename S, bool FIRST, bool FLOOD = false, bool WARM = false>
__global__ __launch_bounds__(64) void k_bp_class(DevPool p, const int4* recs, int nitems, int cls,
                                                 const int32_t* gate) {
    static_assert(!WARM || FIRST, "warm-start messages exist only in a first sweep");
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int G = 2 * C3;
    constexpr int M2 = CHI * CHI;
    constexpr int DPW = BPLayout<CHI>::DPW;
    constexpr int DL = BPLayout<CHI>::DL;
    constexpr int EPG = BPLayout<CHI>::EPG;
    constexpr int MPL = BPRegs<CHI, S>::MPL;
    constexpr bool GREG = BPRegs<CHI, S>::GREG;
    static_assert(3 * CHI <= DL && M2 >= DL && M2 % DL == 0, "direction layout");
    static_assert(C3 % DL == 0, "tensor halves split evenly over the lanes");
    using W = cpx<S>;
    __shared__ W Th[DPW][C3];               // one physical half of T at a time
    __shared__ W Yh[DPW][C3];
    __shared__ W m1[DPW][M2];
    __shared__ W m2[DPW][M2];
    __shared__ double sq[DPW][3][CHI];
    __shared__ double lamv[DPW][3][CHI];
    __shared__ double bnd[DPW][2];

    const int g = wg_index(p.xcd_remap);
    if (g * EPG >= nitems) return;             // uniform over the work-group
    if (gate && *gate == 0) return;            // uniform
    const int lane = threadIdx.x;
    const int d = lane / DL;                   // direction slot
    const int hl = lane % DL;

    BPRegs<CHI, S> ld;
    {
        int4 md, es;
        bp_record<CHI>(recs, nitems, g, d, md, es);
        bp_load<CHI, S, FIRST, FLOOD>(p, md, es, d, hl, cls, ld);
    }
    // A direction without work (item past the end, slot inactive or done)
    // computes on the work-group's first item and stores nothing: every lane
    // takes part in every barrier.
    // (a slot whose stop test waits for the exact distance sweeps no further)
    const bool valid = g * EPG + d / 2 < nitems && (ld.fl & FLAG_ACTIVE) && !(ld.fl & (FLAG_BP_DONE | FLAG_UNDECIDED));
    if (__ballot(valid) == 0) return;          // uniform
    const int e = ld.e;
    const int pleg = ld.md.w & 3;
    int o1, o2;
    other_legs(pleg, o1, o2);
    const int sp = leg_stride<CHI>(pleg), s1 = leg_stride<CHI>(o1), s2 = leg_stride<CHI>(o2);
    if (hl < 3 * CHI) {
        sq[d][hl / CHI][hl % CHI] = sqrt(ld.lv);
        lamv[d][hl / CHI][hl % CHI] = ld.lv;
    }
    __syncthreads();
    // warm-start message diag(lambda)/sum(lambda) of leg lg, entry idx
    auto warm = [&](int lg, int idx) -> S {
        const int r = idx / CHI, c = idx % CHI;
        if (r != c) return S(0);
        double tot = 0.0;
#pragma unroll
        for (int j = 0; j < CHI; ++j) tot += lamv[d][lg][j];
        return S(tot > 0.0 ? lamv[d][lg][r] / tot : 0.0);
    };
    // incoming messages; in the first sweep those of classes not yet
    // visited are the warm start
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const int inc = w == 0 ? ld.md.y : ld.md.z;
        const int col = (ld.md.w >> (8 + 8 * w)) & 255;
        const bool wm = inc >= 0 && FIRST && (FLOOD || col > cls);
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const int idx = hl + DL * k;
            W val = ld.mreg[w][k];
            if (inc < 0) val = {S(idx == 0 ? 1 : 0), S(0)};
            else if (wm) val = {warm(w == 0 ? o1 : o2, idx), S(0)};
            if (w == 0) m1[d][idx] = val;
            else m2[d][idx] = val;
        }
    }
    // the iterate this sweep replaces: the stored message, or in the
    // first sweep the warm start as the iteration used it
    W oldv[MPL];
#pragma unroll
    for (int k = 0; k < MPL; ++k) oldv[k] = FIRST ? W{warm(pleg, hl + DL * k), S(0)} : ld.oldr[k];
    const W* gsrc = reinterpret_cast<const W*>(p.gam) + (size_t)ld.md.x * G;
    // The two physical halves i of T go through LDS one after the
    // other (half the LDS per direction, so more work-groups in
    // flight): Y_i[j][k'][l] = sum_k T[i, j@p, k@o1, l@o2] m1[k][k'],
    // then in place Z_i[j][k'][l'] = sum_l Y_i[j][k'][l] m2[l][l'],
    // and out[j][j'] += sum_{k',l'} Z_i[j][k'][l'] conj(T[i, j'@p, k'@o1, l'@o2]).
    cd tot[MPL];
#pragma unroll
    for (int k = 0; k < MPL; ++k) tot[k] = cz<double>();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if (i) __syncthreads();         // the first half's reads are done
        if (GREG) {
#pragma unroll
            for (int k = i * (C3 / DL); k < (i + 1) * (C3 / DL); ++k) {
                const int idx = hl + DL * k - i * C3;
                const int j0 = idx / (CHI * CHI), j1 = (idx / CHI) % CHI, j2 = idx % CHI;
                const S sc = S(sq[d][0][j0] * sq[d][1][j1] * sq[d][2][j2]);
                Th[d][idx] = {ld.greg[k].re * sc, ld.greg[k].im * sc};
            }
        } else {
            for (int idx = hl; idx < C3; idx += DL) {
                const int j0 = idx / (CHI * CHI), j1 = (idx / CHI) % CHI, j2 = idx % CHI;
                const S sc = S(sq[d][0][j0] * sq[d][1][j1] * sq[d][2][j2]);
                const W gv = gsrc[i * C3 + idx];
                Th[d][idx] = {gv.re * sc, gv.im * sc};
            }
        }
        __syncthreads();
        if constexpr (M2 == DL && CHI == 4) {
            // One row per lane throughout.  Y row (j, l) with l = q; the 4 x 4
            // transpose within the row group's four lanes by quad DPP (lane q
            // sends Y[j][q ^ s][q] to lane q ^ s); then Z row (j, k') with
            // k' = q, kept in registers: the lane forms its k' share of
            // out[j][j'] for every j', the four lanes of row j sum them, and
            // lane j CHI + j' keeps out[j][j'].
            const int j = hl / CHI, q = hl % CHI;
            W acc[CHI];
            {
                const W* tb = &Th[d][j * sp + q * s2];
                if constexpr (WARM) {
#pragma unroll
                    for (int kp = 0; kp < CHI; ++kp) {
                        const W tv = tb[kp * s1];
                        const S dv = m1[d][kp * CHI + kp].re;
                        acc[kp] = {tv.re * dv, tv.im * dv};
                    }
                } else {
#pragma unroll
                    for (int kp = 0; kp < CHI; ++kp) acc[kp] = cz<S>();
#pragma unroll
                    for (int k = 0; k < CHI; ++k) {
                        const W tv = tb[k * s1];
#pragma unroll
                        for (int kp = 0; kp < CHI; ++kp) acc[kp] = cfma(acc[kp], tv, m1[d][k * CHI + kp]);
                    }
                }
            }
            W yv[CHI];                          // yv[s] = Y[j][q][q ^ s]
#pragma unroll
            for (int sx = 0; sx < CHI; ++sx) {
                W send = acc[0];
#pragma unroll
                for (int c = 1; c < CHI; ++c) {
                    if ((q ^ sx) == c) send = acc[c];
                }
                yv[sx] = wxor(send, sx);
            }
            // z[t] = Z[j][k' = q][l' = lz(t)]: lz(t) = t, or with a diagonal m2
            // (WARM) lz(t) = q ^ t, which keeps every register index static
            W z[CHI];
#pragma unroll
            for (int lp = 0; lp < CHI; ++lp) {
                if constexpr (WARM) {
                    const int l = q ^ lp;
                    const S dv = m2[d][l * CHI + l].re;
                    z[lp] = {yv[lp].re * dv, yv[lp].im * dv};
                } else {
                    W a2 = cz<S>();
#pragma unroll
                    for (int sx = 0; sx < CHI; ++sx) a2 = cfma(a2, yv[sx], m2[d][(q ^ sx) * CHI + lp]);
                    z[lp] = a2;
                }
            }
            W mine = cz<S>();
#pragma unroll
            for (int jq = 0; jq < CHI; ++jq) {
                W part = cz<S>();
#pragma unroll
                for (int lp = 0; lp < CHI; ++lp) {
                    const int lz = WARM ? (q ^ lp) : lp;
                    part = cfmac(part, z[lp], Th[d][jq * sp + q * s1 + lz * s2]);
                }
                part = seg_sum<CHI>(part);
                if (jq == q) mine = part;
            }
            tot[0] = cadd(tot[0], to_cd(mine));
            continue;
        }
        if constexpr (WARM) {
            // both incoming messages diagonal: Y[j][k'][l'] = T[j][k'][l'] m1[k'][k'] m2[l'][l']
            // (the values the two full products give), one pass
            for (int rw = hl; rw < M2; rw += DL) {  // rows (j, l)
                const int j = rw / CHI, ll = rw % CHI;
                const W* tb = &Th[d][j * sp + ll * s2];
                const S d2 = m2[d][ll * CHI + ll].re;
#pragma unroll
                for (int kp = 0; kp < CHI; ++kp) {
                    const W tv = tb[kp * s1];
                    const S d1 = m1[d][kp * CHI + kp].re;
                    const W y = {tv.re * d1, tv.im * d1};
                    Yh[d][j * M2 + kp * CHI + ll] = {y.re * d2, y.im * d2};
                }
            }
            __syncthreads();
        } else {
        for (int rw = hl; rw < M2; rw += DL) {      // rows (j, l)
            const int j = rw / CHI, ll = rw % CHI;
            const W* tb = &Th[d][j * sp + ll * s2];
            W acc[CHI];
#pragma unroll
            for (int kp = 0; kp < CHI; ++kp) acc[kp] = cz<S>();
#pragma unroll
            for (int k = 0; k < CHI; ++k) {
                const W tv = tb[k * s1];
#pragma unroll
                for (int kp = 0; kp < CHI; ++kp) acc[kp] = cfma(acc[kp], tv, m1[d][k * CHI + kp]);
            }
#pragma unroll
            for (int kp = 0; kp < CHI; ++kp) Yh[d][j * M2 + kp * CHI + ll] = acc[kp];
        }
        __syncthreads();
        for (int rw = hl; rw < M2; rw += DL) {      // rows (j, k'), in place
            W* yr = &Yh[d][rw * CHI];
            W yv[CHI];
#pragma unroll
            for (int ll = 0; ll < CHI; ++ll) yv[ll] = yr[ll];
#pragma unroll
            for (int lp = 0; lp < CHI; ++lp) {
                W acc = cz<S>();
#pragma unroll
                for (int ll = 0; ll < CHI; ++ll) acc = cfma(acc, yv[ll], m2[d][ll * CHI + lp]);
                yr[lp] = acc;
            }
        }
        __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const int o = hl + DL * k;
            const int j = o / CHI, jp = o % CHI;
            W part = cz<S>();
            for (int kp = 0; kp < CHI; ++kp) {
#pragma unroll
                for (int lp = 0; lp < CHI; ++lp) {
                    part = cfmac(part, Yh[d][j * M2 + kp * CHI + lp], Th[d][jp * sp + kp * s1 + lp * s2]);
                }
            }
            tot[k] = cadd(tot[k], to_cd(part));
        }
    }
    // unit trace, store; bounds on the trace norm of (new - old)
    {
        // unit trace by the complex trace: normalising by its real part
        // only leaves a complex scale that the next sweeps' products compound
        cd tr = cz<double>();
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            if ((hl + DL * k) % (CHI + 1) == 0) tr = cadd(tr, tot[k]);   // diagonal entries
        }
        tr = seg_sum<DL>(tr);
        const double t2 = cabs2(tr);
        const double it2 = t2 > 0.0 ? 1.0 / t2 : 0.0;
        const cd itr = {tr.re * it2, -tr.im * it2};
        W* dst = reinterpret_cast<W*>(p.msg) + ((size_t)e * 2 + (d & 1)) * M2;
        W* mo = reinterpret_cast<W*>(p.mold) + ((size_t)e * 2 + (d & 1)) * M2;
        double f2 = 0.0, l1 = 0.0;
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const int o = hl + DL * k;
            const W nvs = from_cd<S>(cmul(tot[k], itr));
            const cd df = csub(to_cd(nvs), to_cd(oldv[k]));
            if (valid) {
                dst[o] = nvs;
                if (!FLOOD || FIRST) mo[o] = oldv[k];    // flooding: mold already holds it
            }
            const double a2 = cabs2(df);
            f2 += a2;
            l1 += sqrt(a2);
        }
        f2 = seg_sum<DL>(f2);
        l1 = seg_sum<DL>(l1);
        if (hl == 0) {
            const double fro = sqrt(f2);
            bnd[d][0] = fro;
            bnd[d][1] = fmin(sqrt((double)CHI) * fro, l1);
        }
    }
    __syncthreads();
    if (hl == 0 && (d & 1) == 0 && valid) {
        p.edlo[e] = bnd[d][0] + bnd[d + 1][0];
        p.edist[e] = bnd[d][1] + bnd[d + 1][1];
    }
}

// Exact trace norms of the last sweep's differences (new message minus the
// one it replaced) for the edges of undecided slots: the sum of the singular
// values of the Hermitian difference (= sum |eigenvalues|), one lane team
// per direction.
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_bp_exact(DevPool p, const int32_t* items, int nitems, int force) {
    constexpr int M2 = CHI * CHI;
    constexpr int TT = (M2 < 32) ? M2 : 32;
    constexpr int LPC = JLayout<CHI, TT>::LPC;
    constexpr int EPL = JLayout<CHI, TT>::EPL;
    __shared__ double dist[2];
    const int item = blockIdx.x;
    if (item >= nitems) return;
    const int e = items[item];
    const int fl = p.sflag[p.eslot[e]];
    if (!(fl & FLAG_UNDECIDED) && !(force && (fl & FLAG_ACTIVE))) return;
    const int lane = threadIdx.x;
    const int d = lane >> 5;
    const int hl = lane & 31;
    const int tl = hl % TT;
    const int col = JLayout<CHI, TT>::col(tl), g = JLayout<CHI, TT>::grp(tl);
    const cpx<S>* nw = reinterpret_cast<const cpx<S>*>(p.msg) + ((size_t)e * 2 + d) * M2;
    const cpx<S>* od = reinterpret_cast<const cpx<S>*>(p.mold) + ((size_t)e * 2 + d) * M2;
    cd mloc[EPL], vdummy[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int o = (g + LPC * k) * CHI + col;
        mloc[k] = csub(to_cd(nw[o]), to_cd(od[o]));    // exact: both in S, difference in FP64
    }
    jacobi_svd_team<CHI, TT, false>(mloc, vdummy, tl, JACOBI_TOL, JACOBI_MAX_SWEEPS);
    double nrm = 0.0;
#pragma unroll
    for (int k = 0; k < EPL; ++k) nrm += cabs2(mloc[k]);
    nrm = strided_sum<CHI, LPC>(nrm);
    double sv = (g == 0) ? sqrt(nrm) : 0.0;
    sv = seg_sum<TT>(sv);
    if (hl == 0) dist[d] = sv;
    __syncthreads();
    if (lane == 0) p.edexact[e] = dist[0] + dist[1];
}

// fixed-order sum over a slot's edges of x[e] (256 lanes: strided partial
// sums, a butterfly within each wavefront, the four wavefront sums in a fixed
// order); the result is valid in every lane
__device__ double slot_sum(const double* x, int e0, int ne, double* red) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < ne; k += 256) acc += x[e0 + k];
    acc = seg_sum<64>(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

// Per-slot distance bounds and the stop decision where the bounds settle it.
// Counters: [0] += slots still sweeping, [1] += slots whose bounds straddle
// the tolerance (they wait, sweeping no further, until the exact pass
// decides them), [2] += slots that reached max_sweeps unconverged (stopped,
// flagged FLAG_BP_CAPPED), [3] = max over converged slots of
// kSweepBias - sweeps (the fewest sweeps a slot needed).  A slot thus takes
// exactly the sweeps and decisions of one read-back per sweep however many
// sweeps are enqueued between read-backs.
__global__ __launch_bounds__(256) void k_bp_reduce(DevPool p, const int32_t* slots, int nslots,
                                                   int32_t* counters, int force_exact, int max_sweeps) {
    __shared__ double red[256];
    const int s = slots[blockIdx.x];
    const int fl = p.sflag[s];
    if (!(fl & FLAG_ACTIVE) || (fl & (FLAG_BP_DONE | FLAG_UNDECIDED))) return;
    const int e0 = p.s_e0[s], ne = p.s_ne[s];
    const double hi = slot_sum(p.edist, e0, ne, red);
    const double lo = slot_sum(p.edlo, e0, ne, red);
    if (threadIdx.x == 0) {
        const double inv = ne > 0 ? 1.0 / ne : 0.0;
        const int sw = p.ssweeps[s] + 1;
        p.ssweeps[s] = sw;
        p.stot[2 * s] += 1;
        const double tol = p.bp_tol;
        if (force_exact || (tol > 0.0 && lo * inv < tol && hi * inv >= tol)) {
            p.sflag[s] = fl | FLAG_UNDECIDED;
            p.sdist[s] = hi * inv;
            atomicAdd(&counters[1], 1);
        } else if (tol > 0.0 && hi * inv < tol) {
            p.sflag[s] = fl | FLAG_BP_DONE;
            p.sdist[s] = hi * inv;
            atomicMax(&counters[3], kSweepBias - sw);
        } else if (tol > 0.0 && sw >= max_sweeps) {
            p.sflag[s] = fl | FLAG_BP_DONE | FLAG_BP_CAPPED;
            p.sdist[s] = lo * inv;
            atomicAdd(&counters[2], 1);
        } else {
            p.sdist[s] = lo * inv;
            atomicAdd(&counters[0], 1);
        }
    }
}

// stop decision from the exact distances of undecided slots (counters as
// k_bp_reduce)
__global__ __launch_bounds__(256) void k_bp_reduce_exact(DevPool p, const int32_t* slots, int nslots,
                                                         int32_t* counters, int force, int max_sweeps) {
    __shared__ double red[256];
    const int s = slots[blockIdx.x];
    const int fl = p.sflag[s];
    if (!(fl & FLAG_UNDECIDED) && !(force && (fl & FLAG_ACTIVE))) return;
    const int e0 = p.s_e0[s], ne = p.s_ne[s];
    const double ex = slot_sum(p.edexact, e0, ne, red);
    if (threadIdx.x == 0) {
        const double da = ne > 0 ? ex / ne : 0.0;
        p.sdist[s] = da;
        const int nf = fl & ~FLAG_UNDECIDED;
        if (p.bp_tol > 0.0 && da < p.bp_tol) {
            p.sflag[s] = nf | FLAG_BP_DONE;
            if (!force) atomicMax(&counters[3], kSweepBias - p.ssweeps[s]);
        } else if (force) {
            p.sflag[s] = nf;
        } else if (p.bp_tol > 0.0 && p.ssweeps[s] >= max_sweeps) {
            p.sflag[s] = nf | FLAG_BP_DONE | FLAG_BP_CAPPED;
            atomicAdd(&counters[2], 1);
        } else {
            p.sflag[s] = nf;
            atomicAdd(&counters[0], 1);
        }
    }
}

// ------------------------------------------------------------------ Alg. 2
// One edge per team of TL lanes (8 at chi = 4, so eight edges share a
// wavefront; 64 at chi = 8); lane t owns the matrix elements u = t + TL q
// (row u / chi, column u % chi).
template <int CHI>
struct CanonLayout {
    static constexpr int TL = CHI <= 4 ? 2 * CHI : CHI * CHI;   // lanes per edge
    static constexpr int TPW = 64 / TL;                          // edges per wavefront
    static constexpr int EPT = CHI * CHI / TL;                   // elements per lane
};
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_canonicalise(DevPool p, const int32_t* items, int nitems) {
    if (tail_gated_off(p)) return;       // uniform: BP has not stopped
    constexpr int M2 = CHI * CHI;
    constexpr int TL = CanonLayout<CHI>::TL;
    constexpr int TPW = CanonLayout<CHI>::TPW;
    constexpr int EPT = CanonLayout<CHI>::EPT;
    static_assert(M2 % TL == 0 && TL >= CHI, "team layout");
    // messages -> Cholesky factors; after the core is formed, U and conj(V)
    // sorted and truncated
    __shared__ cd A[TPW][2][CHI][CHI];
    __shared__ cd Li[TPW][2][CHI][CHI];  // pseudo-inverses of the factors
    __shared__ double sg[TPW][CHI];
    __shared__ int ordr[TPW][CHI];
    __shared__ double lold[TPW][CHI];
    __shared__ double diagmax[TPW][2];

    const int team = threadIdx.x / TL;
    const int t = threadIdx.x % TL;
    const int item = wg_index(p.xcd_remap) * TPW + team;
    const bool valid = item < nitems;
    const int e = valid ? items[item] : 0;
    // the message and lambda loads issue together with the slot-flag load
    const cpx<S>* msg = reinterpret_cast<const cpx<S>*>(p.msg) + (size_t)e * 2 * M2;
    cd mv[2][EPT];
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int q = 0; q < EPT; ++q) mv[w][q] = to_cd(msg[w * M2 + t + TL * q]);
    const double lv = t < CHI ? p.lam[(size_t)e * CHI + t] : 0.0;
    const int slot = p.eslot[e];
    const bool act = valid && (p.sflag[slot] & FLAG_ACTIVE);
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int u = t + TL * q;
            A[team][w][u / CHI][u % CHI] = act ? mv[w][q] : cz<double>();
        }
    if (t < CHI) lold[team][t] = act ? lv : 0.0;
    __syncthreads();
    if constexpr (CHI <= 4) {
        // Lane t factors message w = t / chi in registers (the chi lanes of
        // each message repeat the same arithmetic) and inverts column
        // col = t % chi of its factor, with no LDS round trips in between.
        static_assert(TL == 2 * CHI, "one lane per factor column");
        const int w = t / CHI, col = t % CHI;
        cd L[CHI][CHI];
        double mx = 0.0;
#pragma unroll
        for (int r = 0; r < CHI; ++r) {
#pragma unroll
            for (int c = 0; c <= r; ++c) L[r][c] = A[team][w][r][c];
            mx = fmax(mx, L[r][r].re);
        }
        // Cholesky m = L L^dagger (lower), pivots <= eig_cut * max diag dropped
#pragma unroll
        for (int k = 0; k < CHI; ++k) {
            const double dk = L[k][k].re;
            const bool piv = dk > p.eig_cut * mx;
            const double sk = piv ? sqrt(dk) : 0.0;
#pragma unroll
            for (int r = k; r < CHI; ++r) L[r][k] = piv ? cscale(L[r][k], 1.0 / sk) : cz<double>();
#pragma unroll
            for (int r = k + 1; r < CHI; ++r)
#pragma unroll
                for (int c = k + 1; c <= r; ++c) L[r][c] = csub(L[r][c], cmulc(L[r][k], L[c][k]));
        }
        // column col of the pseudo-inverse by forward substitution (zero
        // pivots give zero rows and columns)
        double rd[CHI];
#pragma unroll
        for (int i = 0; i < CHI; ++i) rd[i] = L[i][i].re != 0.0 ? 1.0 / L[i][i].re : 0.0;
        const bool live = rd[col] != 0.0;
        cd li[CHI];
#pragma unroll
        for (int i = 0; i < CHI; ++i) {
            cd acc = cz<double>();
#pragma unroll
            for (int k = 0; k < i; ++k) {
                if (k >= col) acc = cfma(acc, L[i][k], li[k]);
            }
            li[i] = !live || i < col || rd[i] == 0.0 ? cz<double>() : (i == col ? cd{rd[i], 0.0} : cscale(acc, -rd[i]));
        }
        __syncthreads();                    // every lane has read its message
#pragma unroll
        for (int r = 0; r < CHI; ++r) {
            cd lv_rc = cz<double>();
#pragma unroll
            for (int c = 0; c < CHI; ++c) {
                if (c == col && c <= r) lv_rc = L[r][c];
            }
            A[team][w][r][col] = lv_rc;
            Li[team][w][r][col] = li[r];
        }
        __syncthreads();
    } else {
        if (t < 2) {
            double mx = 0.0;
            for (int j = 0; j < CHI; ++j) mx = fmax(mx, A[team][t][j][j].re);
            diagmax[team][t] = mx;
        }
        __syncthreads();
        // Cholesky m = L L^dagger (lower), pivots <= eig_cut * max diag dropped
        for (int k = 0; k < CHI; ++k) {
            double dk[2];
#pragma unroll
            for (int w = 0; w < 2; ++w) dk[w] = A[team][w][k][k].re;
            __syncthreads();
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                const bool piv = dk[w] > p.eig_cut * diagmax[team][w];
                const double s = piv ? sqrt(dk[w]) : 0.0;
#pragma unroll
                for (int q = 0; q < EPT; ++q) {
                    const int u = t + TL * q, r = u / CHI, c = u % CHI;
                    if (c == k && r >= k) A[team][w][r][k] = piv ? cscale(A[team][w][r][k], 1.0 / s) : cz<double>();
                }
            }
            __syncthreads();
#pragma unroll
            for (int w = 0; w < 2; ++w)
#pragma unroll
                for (int q = 0; q < EPT; ++q) {
                    const int u = t + TL * q, r = u / CHI, c = u % CHI;
                    if (r > k && c > k && c <= r)
                        A[team][w][r][c] = csub(A[team][w][r][c], cmulc(A[team][w][r][k], A[team][w][c][k]));
                }
            __syncthreads();
        }
#pragma unroll
        for (int w = 0; w < 2; ++w)
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const int u = t + TL * q, r = u / CHI, c = u % CHI;
                if (c > r) A[team][w][r][c] = cz<double>();
            }
        __syncthreads();
        // pseudo-inverse of each lower-triangular factor, one column per lane,
        // by forward substitution in registers (zero pivots give zero rows and
        // columns)
        for (int wc = t; wc < 2 * CHI; wc += TL) {
            const int w = wc / CHI, col = wc % CHI;
            double rd[CHI];
            cd lrow[CHI][CHI];
#pragma unroll
            for (int i = 0; i < CHI; ++i) {
                const double di = A[team][w][i][i].re;
                rd[i] = di != 0.0 ? 1.0 / di : 0.0;
#pragma unroll
                for (int k = 0; k < i; ++k) lrow[i][k] = A[team][w][i][k];
            }
            const bool live = rd[col] != 0.0;
            cd li[CHI];
#pragma unroll
            for (int i = 0; i < CHI; ++i) {
                cd acc = cz<double>();
#pragma unroll
                for (int k = 0; k < i; ++k) {
                    if (k >= col) acc = cfma(acc, lrow[i][k], li[k]);
                }
                li[i] = !live || i < col || rd[i] == 0.0 ? cz<double>() : (i == col ? cd{rd[i], 0.0} : cscale(acc, -rd[i]));
            }
#pragma unroll
            for (int i = 0; i < CHI; ++i) Li[team][w][i][col] = li[i];
        }
        __syncthreads();
    }
    // bond core C[k][l] = sum_j L1[j][k] L2[j][l] in the layout of
    // jacobi_svd_team<CHI, TL>: lane t -> column t % CHI, rows g + LPC k (g = t / CHI)
    constexpr int LPC = JLayout<CHI, TL>::LPC;
    constexpr int EPL = JLayout<CHI, TL>::EPL;
    const int jcol = JLayout<CHI, TL>::col(t), jg = JLayout<CHI, TL>::grp(t);
    cd m[EPL], v[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int row = jg + LPC * k;
        cd acc = cz<double>();
        for (int j = 0; j < CHI; ++j) acc = cfma(acc, A[team][0][j][row], A[team][1][j][jcol]);
        m[k] = acc;
        v[k] = (row == jcol) ? cd{1.0, 0.0} : cz<double>();
    }
    const int sweeps = jacobi_svd_team<CHI, TL>(m, v, t, JACOBI_TOL, JACOBI_MAX_SWEEPS);
    if (act && sweeps > JACOBI_MAX_SWEEPS && t == 0) atomicOr(&p.swarn[slot], (int)WARN_JACOBI);
    double nl = 0.0;
#pragma unroll
    for (int k = 0; k < EPL; ++k) nl += cabs2(m[k]);
    nl = strided_sum<CHI, LPC>(nl);
    const double sgm = sqrt(nl);
    if (jg == 0) sg[team][jcol] = sgm;
    if (t < CHI) ordr[team][t] = t;
    __syncthreads();
    if (t < CHI) {
        int rank = 0;
        const double me = sg[team][t];
        for (int k = 0; k < CHI; ++k) {
            const double o = sg[team][k];
            rank += (o > me || (o == me && k < t)) ? 1 : 0;
        }
        if (rank < CHI) ordr[team][rank] = t;
    }
    __syncthreads();
    const double smax = sg[team][ordr[team][0]];
    int rk = 0;
    double kept2 = 0.0;
    for (int k = 0; k < CHI; ++k) {
        const double sk = sg[team][ordr[team][k]];
        if (sk > p.svd_cut * smax) {
            rk = k + 1;
            kept2 += sk * sk;
        }
    }
    // scatter U and conj(V) columns into sorted positions
    {
        int dstq = 0;
        for (int k = 0; k < CHI; ++k) if (ordr[team][k] == jcol) dstq = k;
        const double isg = sgm > 0.0 ? 1.0 / sgm : 0.0;
        const bool keep = dstq < rk;
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int row = jg + LPC * k;
            A[team][0][row][dstq] = keep ? cscale(m[k], isg) : cz<double>();
            A[team][1][row][dstq] = keep ? cconj(v[k]) : cz<double>();
        }
    }
    __syncthreads();
    if (!act) return;
    // X_u[j][q] = sqrt(lambda_old[j]) sum_j' Li1[j'][j] U[j'][q]; same for v with conj(V)
    cpx<S>* xg = reinterpret_cast<cpx<S>*>(p.xg) + (size_t)e * 2 * M2;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int u = t + TL * q, r = u / CHI, c = u % CHI;
        const double sl = sqrt(lold[team][r]);
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            cd acc = cz<double>();
            for (int jp = 0; jp < CHI; ++jp) acc = cfma(acc, Li[team][w][jp][r], A[team][w][jp][c]);
            xg[w * M2 + u] = from_cd<S>(cscale(acc, sl));
        }
    }
    if (t < CHI) {
        const double inv = kept2 > 0.0 ? 1.0 / sqrt(kept2) : 0.0;
        p.lam[(size_t)e * CHI + t] = t < rk ? sg[team][ordr[team][t]] * inv : 0.0;
    }
}

// Alg. 2 at chi = 4 with one lane per column of the bond core, sixteen edges
// per wavefront.  Each lane factors both messages and inverts both factors
// in registers (the four lanes of an edge repeat that arithmetic, as the
// eight-lane team did), forms its column of the core C = L1^T L2, and the
// four-lane team Jacobi then holds a whole column per lane: rotations need
// only quad DPP moves and no cross-lane sum.  The sorted U and conj(V)
// columns are gathered from the lane of the right rank, and each lane writes
// its column of both gauge maps.  Same pivot rule, cutoffs, Jacobi and
// ordering as k_canonicalise.  (Recomputing the factors after the Jacobi
// instead of holding their inverses, for four wavefronts per SIMD instead of
// two, measured slower: 146 against 126 us per launch of 384,000 edges.)
template <typename S>
__global__ __launch_bounds__(64) void k_canonicalise4(DevPool p, const int32_t* items, int nitems) {
    if (tail_gated_off(p)) return;       // uniform: BP has not stopped
    constexpr int CHI = 4;
    constexpr int M2 = CHI * CHI;
    const int lane = threadIdx.x;
    const int team = lane >> 2, q = lane & 3;
    const int item = wg_index(p.xcd_remap) * 16 + team;
    const bool valid = item < nitems;
    const int e = items[valid ? item : 0];
    const cpx<S>* msg = reinterpret_cast<const cpx<S>*>(p.msg) + (size_t)e * 2 * M2;
    cd L[2][CHI][CHI];
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int r = 0; r < CHI; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) L[w][r][c] = to_cd(msg[w * M2 + r * CHI + c]);
    double lold[CHI];
#pragma unroll
    for (int j = 0; j < CHI; ++j) lold[j] = p.lam[(size_t)e * CHI + j];
    const int slot = p.eslot[e];
    const bool act = valid && (p.sflag[slot] & FLAG_ACTIVE);
    // Cholesky m = L L^dagger (lower), pivots <= eig_cut * max diag dropped
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        double mx = 0.0;
#pragma unroll
        for (int r = 0; r < CHI; ++r) mx = fmax(mx, L[w][r][r].re);
#pragma unroll
        for (int k = 0; k < CHI; ++k) {
            const double dk = L[w][k][k].re;
            const bool piv = dk > p.eig_cut * mx;
            const double sk = piv ? sqrt(dk) : 0.0;
#pragma unroll
            for (int r = k; r < CHI; ++r) L[w][r][k] = piv ? cscale(L[w][r][k], 1.0 / sk) : cz<double>();
#pragma unroll
            for (int r = k + 1; r < CHI; ++r)
#pragma unroll
                for (int c = k + 1; c <= r; ++c) L[w][r][c] = csub(L[w][r][c], cmulc(L[w][r][k], L[w][c][k]));
        }
    }
    // column q of the core, C[k][q] = sum_j L1[j][k] L2[j][q]
    cd m[CHI], v[CHI];
#pragma unroll
    for (int k = 0; k < CHI; ++k) {
        cd acc = cz<double>();
#pragma unroll
        for (int j = 0; j < CHI; ++j) {
            cd l2 = cz<double>();
#pragma unroll
            for (int c = 0; c < CHI; ++c)
                if (c == q && j >= c) l2 = L[1][j][c];
            if (j >= k) acc = cfma(acc, L[0][j][k], l2);
        }
        m[k] = acc;
        v[k] = (k == q) ? cd{1.0, 0.0} : cz<double>();
    }
    // pseudo-inverses of the factors, by forward substitution (zero pivots
    // give zero rows and columns); Li[w][i][col]
    cd Li[2][CHI][CHI];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        double rd[CHI];
#pragma unroll
        for (int i = 0; i < CHI; ++i) rd[i] = L[w][i][i].re != 0.0 ? 1.0 / L[w][i][i].re : 0.0;
#pragma unroll
        for (int col = 0; col < CHI; ++col) {
            const bool live = rd[col] != 0.0;
#pragma unroll
            for (int i = 0; i < CHI; ++i) {
                cd acc = cz<double>();
#pragma unroll
                for (int k = col; k < i; ++k) acc = cfma(acc, L[w][i][k], Li[w][k][col]);
                Li[w][i][col] = !live || i < col || rd[i] == 0.0 ? cz<double>()
                                                                : (i == col ? cd{rd[i], 0.0} : cscale(acc, -rd[i]));
            }
        }
    }
    const int sweeps = jacobi_svd_team<CHI, 4>(m, v, q, JACOBI_TOL, JACOBI_MAX_SWEEPS);
    if (act && sweeps > JACOBI_MAX_SWEEPS && q == 0) atomicOr(&p.swarn[slot], (int)WARN_JACOBI);
    double n2 = 0.0;
#pragma unroll
    for (int k = 0; k < CHI; ++k) n2 += cabs2(m[k]);
    const double sgm = sqrt(n2);
    // rank of this column (descending, ties by column index), the number of
    // values above the cutoff and their squared sum
    int rank = 0, rk = 0;
    double smax = sgm;
#pragma unroll
    for (int r = 1; r < CHI; ++r) smax = fmax(smax, xshfl(sgm, r));
    double kept2 = 0.0;
#pragma unroll
    for (int r = 0; r < CHI; ++r) {
        const double o = r ? xshfl(sgm, r) : sgm;
        if (r) rank += (o > sgm || (o == sgm && (q ^ r) < q)) ? 1 : 0;
        if (o > p.svd_cut * smax) {
            ++rk;
            kept2 += o * o;
        }
    }
    // this lane takes the column of rank q (and its sigma)
    cd us[CHI], vs[CHI];
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < CHI; ++r) {
        const int ro = r ? xshfl_i(rank, r) : rank;
        const bool take = ro == q;
        const double so = r ? xshfl(sgm, r) : sgm;
        if (take) ss = so;
#pragma unroll
        for (int k = 0; k < CHI; ++k) {
            const cd mo = r ? shfl_xor_cd(m[k], r) : m[k];
            const cd vo = r ? shfl_xor_cd(v[k], r) : v[k];
            if (take) {
                us[k] = mo;
                vs[k] = vo;
            }
        }
    }
    if (!act) return;
    const bool keep = q < rk;
    const double isg = (keep && ss > 0.0) ? 1.0 / ss : 0.0;
    // X_u[j][q] = sqrt(lambda_old[j]) sum_j' Li1[j'][j] U[j'][q]; X_v with conj(V)
    cpx<S>* xg = reinterpret_cast<cpx<S>*>(p.xg) + (size_t)e * 2 * M2;
#pragma unroll
    for (int j = 0; j < CHI; ++j) {
        const double sl = sqrt(lold[j]);
        cd au = cz<double>(), av = cz<double>();
#pragma unroll
        for (int jp = 0; jp < CHI; ++jp) {
            au = cfma(au, Li[0][jp][j], keep ? cscale(us[jp], isg) : cz<double>());
            av = cfma(av, Li[1][jp][j], keep ? cconj(vs[jp]) : cz<double>());
        }
        xg[j * CHI + q] = from_cd<S>(cscale(au, sl));
        xg[M2 + j * CHI + q] = from_cd<S>(cscale(av, sl));
    }
    const double inv = kept2 > 0.0 ? 1.0 / sqrt(kept2) : 0.0;
    p.lam[(size_t)e * CHI + q] = keep ? ss * inv : 0.0;
}

// ------------------------------------------------------------------ gauge apply + X
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_gauge_apply(DevPool p, const int32_t* items, int nitems,
                                                    int apply_x_allowed) {
    if (tail_gated_off(p)) return;       // uniform: BP has not stopped
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int G = 2 * C3;
    constexpr int M2 = CHI * CHI;
    using W = cpx<S>;
    // The gauge maps act on the virtual legs only, so at chi = 8 the two
    // physical halves go through LDS one after the other (half the LDS per
    // vertex: 4 wavefronts per SIMD instead of 2); at chi = 4 the whole
    // tensor fits and one pass is faster.
    constexpr int NH = CHI > 4 ? 2 : 1;     // passes
    constexpr int HS = G / NH;              // elements per pass
    __shared__ W buf[2][HS];
    __shared__ W X[3][M2];

    const int item = wg_index(p.xcd_remap);
    if (item >= nitems) return;
    const int a = items[item];
    const int lane = threadIdx.x;
    // gauge maps and the tensor load one level after the metadata, with the flag
    const int4 vm = p.vmeta[a];
    const int slot = vm.w;
    W* gam = reinterpret_cast<W*>(p.gam) + (size_t)a * G;
    constexpr int XPL = (3 * M2 + 63) / 64;
    W xr[XPL];
#pragma unroll
    for (int k = 0; k < XPL; ++k) {
        const int idx = lane + 64 * k;
        const int lg = idx / M2, o = idx % M2;
        W val = cz<S>();
        if (idx < 3 * M2) {
            const int xi = lg == 0 ? vm.x : (lg == 1 ? vm.y : vm.z);
            if (xi < 0) val = {S(o == 0 ? 1 : 0), S(0)};
            else val = reinterpret_cast<const W*>(p.xg)[(size_t)xi * M2 + o];
        }
        xr[k] = val;
    }
    constexpr int GPL = G / 64;
    constexpr bool GREG = GPL <= 4;
    W gr[GREG ? GPL : 1];
    if (GREG) {
#pragma unroll
        for (int k = 0; k < GPL; ++k) gr[k] = gam[lane + 64 * k];
    }
    const int fl = p.sflag[slot];
    if (!(fl & FLAG_ACTIVE)) return;
#pragma unroll
    for (int k = 0; k < XPL; ++k) {
        const int idx = lane + 64 * k;
        if (idx < 3 * M2) X[idx / M2][idx % M2] = xr[k];
    }
    const bool do_x = apply_x_allowed && (fl & FLAG_APPLY_X);
    S c = S(1), s = S(0);
    if (do_x) {
        double sn, cs;
        sincos(p.theta[2 * slot + 1], &sn, &cs);
        c = S(cs);
        s = S(sn);
    }
    if constexpr (CHI == 4) {
        // Lane t holds entries t (i = 0) and t + 64 (i = 1), whose virtual
        // indices are j0 = t >> 4, j1 = (t >> 2) & 3, j2 = t & 3: the four
        // entries a mode product mixes sit in lanes t ^ (u << sh) (sh = 4, 2, 0
        // for legs 0, 1, 2), so each product runs on cross-lane moves with
        // the maps read from LDS, and U_X acts within the lane.
        __syncthreads();                    // X
        W g[2] = {gr[0], gr[1]};
#pragma unroll
        for (int lg = 0; lg < 3; ++lg) {
            const int sh = lg == 0 ? 4 : (lg == 1 ? 2 : 0);
            const int jown = (lane >> sh) & 3;
            W xk[CHI];
#pragma unroll
            for (int u = 0; u < CHI; ++u) xk[u] = X[lg][(jown ^ u) * CHI + jown];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                W acc = cz<S>();
#pragma unroll
                for (int u = 0; u < CHI; ++u) acc = cfma(acc, wxor(g[e], u << sh), xk[u]);
                g[e] = acc;
            }
        }
        if (!do_x) {
            gam[lane] = g[0];
            gam[C3 + lane] = g[1];
        } else {
            const W g0 = g[0], g1 = g[1];
            gam[lane] = {c * g0.re + s * g1.im, c * g0.im - s * g1.re};
            gam[C3 + lane] = {s * g0.im + c * g1.re, -s * g0.re + c * g1.im};
        }
        return;
    }
    constexpr int HPL = (C3 + 63) / 64;     // elements of a half per lane
    W half0[NH == 2 ? HPL : 1];             // the first half's result, for U_X
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        if (i) __syncthreads();             // the first half's reads are done
        if (GREG) {
            static_assert(!GREG || HS % 64 == 0, "passes split evenly over the lanes");
#pragma unroll
            for (int k = i * (HS / 64); k < (i + 1) * (HS / 64); ++k) buf[0][lane + 64 * k - i * HS] = gr[k];
        } else {
            for (int idx = lane; idx < HS; idx += 64) buf[0][idx] = gam[i * HS + idx];
        }
        __syncthreads();
        // contract legs 0, 1, 2 in turn: out[.. j@l ..] = sum_k in[.. k@l ..] X_l[k][j]
#pragma unroll
        for (int lg = 0; lg < 3; ++lg) {
            const W* in = buf[lg & 1];
            W* out = buf[(lg + 1) & 1];
            const int st = leg_stride<CHI>(lg);
            for (int idx = lane; idx < HS; idx += 64) {
                const int j = (idx / st) % CHI;
                const int base = idx - j * st;
                W acc = cz<S>();
#pragma unroll
                for (int k = 0; k < CHI; ++k) acc = cfma(acc, in[base + k * st], X[lg][k * CHI + j]);
                out[idx] = acc;
            }
            __syncthreads();
        }
        const W* res = buf[1];
        // [c, -i s; -i s, c] on the physical index when U_X is fused
#pragma unroll
        for (int k = 0; k < HPL; ++k) {
            const int idx = lane + 64 * k;
            if (idx >= C3) continue;
            if (NH == 1) {
                const W g0 = res[idx], g1 = res[C3 + idx];
                if (!do_x) {
                    gam[idx] = g0;
                    gam[C3 + idx] = g1;
                } else {
                    gam[idx] = {c * g0.re + s * g1.im, c * g0.im - s * g1.re};
                    gam[C3 + idx] = {s * g0.im + c * g1.re, -s * g0.re + c * g1.im};
                }
            } else if (!do_x) {
                gam[i * C3 + idx] = res[idx];
            } else if (i == 0) {
                half0[k] = res[idx];
            } else {
                const W g0 = half0[k], g1 = res[idx];
                gam[idx] = {c * g0.re + s * g1.im, c * g0.im - s * g1.re};
                gam[C3 + idx] = {s * g0.im + c * g1.re, -s * g0.re + c * g1.im};
            }
        }
    }
}

template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_x_layer(DevPool p, const int32_t* items, int nitems) {
    constexpr int C3 = CHI * CHI * CHI;
    using W = cpx<S>;
    const int item = blockIdx.x;
    if (item >= nitems) return;
    const int a = items[item];
    const int slot = p.vslot[a];
    double sn, cs;
    sincos(p.theta[2 * slot + 1], &sn, &cs);
    const S c = S(cs), s = S(sn);
    W* gam = reinterpret_cast<W*>(p.gam) + (size_t)a * 2 * C3;
    for (int idx = threadIdx.x; idx < C3; idx += 64) {
        const W g0 = gam[idx], g1 = gam[C3 + idx];
        gam[idx] = {c * g0.re + s * g1.im, c * g0.im - s * g1.re};
        gam[C3 + idx] = {s * g0.im + c * g1.re, -s * g0.re + c * g1.im};
    }
}

// ------------------------------------------------------------------ readout
// rho_a[i][i'] ~ sum_J Gamma[i][J] conj(Gamma[i'][J]) prod lambda^2 (Vidal form)
// or ~ sum T[i,J] conj(T[i',J']) prod m (message form, Eq. partial_dens).
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_readout(DevPool p, const int32_t* items, int nitems,
                                                int from_messages) {
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int M2 = CHI * CHI;
    using W = cpx<S>;
    __shared__ double wl[3][CHI];
    __shared__ cd Ms[3][M2];
    __shared__ cd Tl[2][C3];
    const int item = blockIdx.x;
    if (item >= nitems) return;
    const int a = items[item];
    const int lane = threadIdx.x;
    const W* gam = reinterpret_cast<const W*>(p.gam) + (size_t)a * 2 * C3;
    cd r00 = cz<double>(), r11 = cz<double>(), r01 = cz<double>();
    if (!from_messages) {
        for (int idx = lane; idx < 3 * CHI; idx += 64) {
            const double lv = leg_lambda(p, a, idx / CHI, idx % CHI, CHI);
            wl[idx / CHI][idx % CHI] = lv * lv;
        }
        __syncthreads();
        for (int idx = lane; idx < C3; idx += 64) {
            const int j0 = idx / M2, j1 = (idx / CHI) % CHI, j2 = idx % CHI;
            const double w = wl[0][j0] * wl[1][j1] * wl[2][j2];
            const cd g0 = to_cd(gam[idx]), g1 = to_cd(gam[C3 + idx]);
            r00.re += w * cabs2(g0);
            r11.re += w * cabs2(g1);
            r01 = cadd(r01, cscale(cmulc(g0, g1), w));
        }
    } else {
        for (int idx = lane; idx < 3 * CHI; idx += 64) {
            wl[idx / CHI][idx % CHI] = sqrt(leg_lambda(p, a, idx / CHI, idx % CHI, CHI));
        }
        for (int idx = lane; idx < 3 * M2; idx += 64) {
            const W* in = incoming_msg<S>(p, a, idx / M2, CHI);
            const int o = idx % M2;
            Ms[idx / M2][o] = in ? to_cd(in[o]) : cd{o == 0 ? 1.0 : 0.0, 0.0};
        }
        __syncthreads();
        for (int idx = lane; idx < 2 * C3; idx += 64) {
            const int j0 = (idx / M2) % CHI, j1 = (idx / CHI) % CHI, j2 = idx % CHI;
            Tl[idx / C3][idx % C3] = cscale(to_cd(gam[idx]), wl[0][j0] * wl[1][j1] * wl[2][j2]);
        }
        __syncthreads();
        // rho[i][i'] = sum_{J,J'} T[i][J] conj(T[i'][J']) m0[j0][j0'] m1[j1][j1'] m2[j2][j2']
        for (int idx = lane; idx < C3; idx += 64) {
            const int j0 = idx / M2, j1 = (idx / CHI) % CHI, j2 = idx % CHI;
            cd s0 = cz<double>(), s1 = cz<double>();   // sum_{J'} m(J,J') conj(T[i'][J'])
            for (int q = 0; q < C3; ++q) {
                const int k0 = q / M2, k1 = (q / CHI) % CHI, k2 = q % CHI;
                const cd w = cmul(cmul(Ms[0][j0 * CHI + k0], Ms[1][j1 * CHI + k1]), Ms[2][j2 * CHI + k2]);
                s0 = cfmac(s0, w, Tl[0][q]);
                s1 = cfmac(s1, w, Tl[1][q]);
            }
            r00 = cfma(r00, Tl[0][idx], s0);
            r11 = cfma(r11, Tl[1][idx], s1);
            r01 = cfma(r01, Tl[0][idx], s1);
        }
    }
    r00 = seg_sum<64>(r00);
    r11 = seg_sum<64>(r11);
    r01 = seg_sum<64>(r01);
    if (lane == 0) {
        const double tr = r00.re + r11.re;
        const double it = tr != 0.0 ? 1.0 / tr : 0.0;
        double* out = p.rho + (size_t)a * 8;
        out[0] = r00.re * it; out[1] = 0.0;
        out[2] = r01.re * it; out[3] = r01.im * it;
        out[4] = r01.re * it; out[5] = -r01.im * it;
        out[6] = r11.re * it; out[7] = 0.0;
        p.zval[a] = (r00.re - r11.re) * it;
        p.xbits[a] = (r00.re * it > 0.5) ? int8_t(1) : int8_t(-1);
    }
}

__global__ __launch_bounds__(256) void k_energy(DevPool p, const int32_t* slots, int nslots) {
    __shared__ double red[256];
    const int s = slots[blockIdx.x];
    const int e0 = p.s_e0[s], ne = p.s_ne[s], v0 = p.s_v0[s], nv = p.s_nv[s];
    double acc = 0.0;
    for (int k = threadIdx.x; k < ne; k += 256) {
        const int e = e0 + k;
        acc += p.J[e] * double(p.xbits[p.eend[2 * e]]) * double(p.xbits[p.eend[2 * e + 1]]);
    }
    for (int k = threadIdx.x; k < nv; k += 256) acc += p.h[v0 + k] * double(p.xbits[v0 + k]);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) p.senergy[s] = red[0];
}

__global__ void k_phase_flags(DevPool p, const int32_t* slots, int n, int phase, int32_t* clear4) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (clear4 && i < 4) clear4[i] = 0;     // the stop-test counters of the re-gauging to come
    if (i >= n) return;
    const int s = slots[i];
    int fl;
    if (phase < 0) {
        fl = FLAG_ACTIVE | FLAG_APPLY_X;
    } else {
        const int mask = p.smask[s];
        fl = ((mask >> phase) & 1) ? FLAG_ACTIVE : 0;
        if ((fl & FLAG_ACTIVE) && (mask >> (phase + 1)) == 0) fl |= FLAG_APPLY_X;
    }
    p.sflag[s] = fl;
    p.ssweeps[s] = 0;
    p.sdist[s] = 0.0;
    if (fl & FLAG_ACTIVE) p.stot[2 * s + 1] += 1;
}

// ------------------------------------------------------------------ Vidal residual (App. C)
// Per vertex a and real leg b: M[j][j'] = sum Gamma_a[.., j@b, ..] conj(Gamma_a[.., j'@b, ..])
// prod_{c != b} lambda_ca^2; with d = bond dimension of b, the term is the
// trace norm of D = delta_d - (d / tr M) M (M compared with the identity
// after division by its mean eigenvalue, since Alg. 2 fixes Gamma_a only up
// to a positive scale).  A group of LPV = chi^2 lanes handles one vertex.
template <int CHI>
struct ResLayout {
    static constexpr int LPV = CHI * CHI;          // lanes per vertex
    static constexpr int VPW = 64 / LPV;           // vertices per wavefront
    static constexpr int NT = CHI * (CHI + 1) / 2; // Gram entries j <= j' per leg
};

// Loads Gamma_a, the squared lambdas and bond dimensions of a's legs, and
// forms the three Gram matrices M (zero outside the bond dimension).
// Lanes vl = 0 .. LPV-1 of the vertex's group share the work.
template <int CHI, typename S, int LPV>
__device__ void residual_grams(const DevPool& p, int a, int vl, cpx<S>* G, double (*lam2)[CHI], int* dims,
                               cd (*Mm)[CHI * CHI]) {
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int NT = ResLayout<CHI>::NT;
    const cpx<S>* gam = reinterpret_cast<const cpx<S>*>(p.gam) + (size_t)a * 2 * C3;
    for (int idx = vl; idx < 2 * C3; idx += LPV) G[idx] = gam[idx];
    for (int idx = vl; idx < 3 * CHI; idx += LPV) {
        const double lv = leg_lambda(p, a, idx / CHI, idx % CHI, CHI);
        lam2[idx / CHI][idx % CHI] = lv * lv;
    }
    if (vl < 3) {
        const int e2 = p.vedge[3 * a + vl];
        int dim = 0;
        if (e2 >= 0)
            for (int j = 0; j < CHI; ++j)
                if (p.lam[(size_t)e2 * CHI + j] > 0.0) dim = j + 1;
        dims[vl] = dim;
    }
    __syncthreads();
    for (int t = vl; t < 3 * NT; t += LPV) {
        const int lg = t / NT;
        int rem = t % NT, j = 0;
        while (rem >= CHI - j) {
            rem -= CHI - j;
            ++j;
        }
        const int jp = j + rem;
        cd acc = cz<double>();
        if (jp < dims[lg]) {
            int o1, o2;
            other_legs(lg, o1, o2);
            const int sb = leg_stride<CHI>(lg), s1 = leg_stride<CHI>(o1), s2 = leg_stride<CHI>(o2);
            cd acc2 = cz<double>();
            for (int i = 0; i < 2; ++i)
#pragma unroll 2
                for (int k1 = 0; k1 < CHI; ++k1) {
                    const double w1 = lam2[o1][k1];
#pragma unroll
                    for (int k2 = 0; k2 < CHI; k2 += 2) {
                        const int b0 = i * C3 + k1 * s1 + k2 * s2;
                        const int b1 = b0 + s2;
                        acc = cadd(acc, cscale(cmulc(to_cd(G[b0 + j * sb]), to_cd(G[b0 + jp * sb])),
                                               w1 * lam2[o2][k2]));
                        acc2 = cadd(acc2, cscale(cmulc(to_cd(G[b1 + j * sb]), to_cd(G[b1 + jp * sb])),
                                                 w1 * lam2[o2][k2 + 1]));
                    }
                }
            acc = cadd(acc, acc2);
        }
        Mm[lg][j * CHI + jp] = acc;
        Mm[lg][jp * CHI + j] = cconj(acc);
    }
    __syncthreads();
}

// D[j][j'] of leg lg from its Gram matrix
template <int CHI>
__device__ __forceinline__ cd residual_d(const cd* Mg, int dim, int j, int jp) {
    double tr = 0.0;
    for (int q = 0; q < CHI; ++q) tr += Mg[q * CHI + q].re;
    const double sc = tr > 0.0 ? dim / tr : 0.0;
    cd dv = cscale(Mg[j * CHI + jp], -sc);
    if (j == jp && j < dim) dv.re += 1.0;
    return dv;
}

// Exact per-vertex sums: the trace norm is the sum of the singular values
// of D (one-sided Jacobi, one team of chi^2 lanes per leg; at chi = 4 the
// three legs run side by side).
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_residual(DevPool p, const int32_t* items, int nitems, int only_undecided) {
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int M2 = CHI * CHI;
    constexpr int TT = M2;                          // team of the chi x chi SVD
    constexpr int LPC = JLayout<CHI, TT>::LPC;
    constexpr int EPL = JLayout<CHI, TT>::EPL;
    constexpr bool PAR = 3 * TT <= 64;
    __shared__ cpx<S> G[2 * C3];
    __shared__ double lam2[3][CHI];
    __shared__ int dims[3];
    __shared__ cd Mm[3][M2];
    __shared__ double term[3];
    const int item = blockIdx.x;
    if (item >= nitems) return;
    const int a = items[item];
    if (only_undecided && !(p.sflag[p.vslot[a]] & FLAG_UNDECIDED)) return;
    const int lane = threadIdx.x;
    residual_grams<CHI, S, 64>(p, a, lane, G, lam2, dims, Mm);
    const int tl = lane % TT;
    const int col = JLayout<CHI, TT>::col(tl), g = JLayout<CHI, TT>::grp(tl);
    constexpr int ROUNDS = PAR ? 1 : 3;
    for (int rd = 0; rd < ROUNDS; ++rd) {
        const int lg = PAR ? ((lane / TT) < 3 ? lane / TT : 0) : rd;
        const int dim = dims[lg];
        cd mloc[EPL], vdummy[EPL];
#pragma unroll
        for (int k = 0; k < EPL; ++k) mloc[k] = residual_d<CHI>(Mm[lg], dim, g + LPC * k, col);
        jacobi_svd_team<CHI, TT, false>(mloc, vdummy, tl, JACOBI_TOL, JACOBI_MAX_SWEEPS);
        double nrm = 0.0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) nrm += cabs2(mloc[k]);
        nrm = strided_sum<CHI, LPC>(nrm);
        double sv = (g == 0) ? sqrt(nrm) : 0.0;
        sv = seg_sum<TT>(sv);
        if (tl == 0 && (PAR ? lane / TT < 3 : true)) term[lg] = dim > 0 ? sv : 0.0;
    }
    __syncthreads();
    if (lane == 0) p.vres[a] = term[0] + term[1] + term[2];
}

// Bounds on the same per-vertex sums without an SVD: for each leg,
// ||D||_F <= ||D||_1 <= min(sqrt(d) ||D||_F, sum_ij |D_ij|).
// At chi <= 4 each leg's Gram matrix is summed in registers: four lanes per
// leg take a quarter of its 2 chi^2 fibres (the vectors over the leg's index
// at fixed other indices) each, so every tensor entry is read from LDS once
// per leg instead of once per Gram entry, and the quad sums by DPP.
template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_residual_bounds(DevPool p, const int32_t* items, int nitems) {
    constexpr int C3 = CHI * CHI * CHI;
    constexpr int M2 = CHI * CHI;
    constexpr int LPV = ResLayout<CHI>::LPV;
    constexpr int VPW = ResLayout<CHI>::VPW;
    __shared__ cpx<S> G[VPW][2 * C3];
    __shared__ double lam2[VPW][3][CHI];
    __shared__ int dims[VPW][3];
    const int lane = threadIdx.x;
    const int sub = lane / LPV, vl = lane % LPV;
    const int item = wg_index(p.xcd_remap) * VPW + sub;
    const bool valid = item < nitems;               // padding groups recompute items[0], write nothing
    const int a = items[valid ? item : 0];
    if constexpr (CHI <= 4) {
        static_assert(LPV == 16, "four lanes for each of the three legs");
        constexpr int NT = ResLayout<CHI>::NT;
        constexpr int NF = 2 * CHI * CHI;            // fibres per leg
        const cpx<S>* gam = reinterpret_cast<const cpx<S>*>(p.gam) + (size_t)a * 2 * C3;
        for (int idx = vl; idx < 2 * C3; idx += LPV) G[sub][idx] = gam[idx];
        for (int idx = vl; idx < 3 * CHI; idx += LPV) {
            const double lv = leg_lambda(p, a, idx / CHI, idx % CHI, CHI);
            lam2[sub][idx / CHI][idx % CHI] = lv * lv;
        }
        if (vl < 3) {
            const int e2 = p.vedge[3 * a + vl];
            int dim = 0;
            if (e2 >= 0)
                for (int j = 0; j < CHI; ++j)
                    if (p.lam[(size_t)e2 * CHI + j] > 0.0) dim = j + 1;
            dims[sub][vl] = dim;
        }
        __syncthreads();
        const int lg = vl / 4 < 3 ? vl / 4 : 2;     // lanes 12..15 repeat leg 2 and contribute nothing
        const int q = vl % 4;
        int o1, o2;
        other_legs(lg, o1, o2);
        const int sb = leg_stride<CHI>(lg), s1 = leg_stride<CHI>(o1), s2 = leg_stride<CHI>(o2);
        // upper triangle of M[j][j'] = sum_fibres w v_j conj(v_j'), row-major
        cd acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = cz<double>();
#pragma unroll 2
        for (int f = q; f < NF; f += 4) {
            const int i = f / M2, k1 = (f / CHI) % CHI, k2 = f % CHI;
            const double w = lam2[sub][o1][k1] * lam2[sub][o2][k2];
            const int base = i * C3 + k1 * s1 + k2 * s2;
            cd v[CHI];
#pragma unroll
            for (int j = 0; j < CHI; ++j) v[j] = to_cd(G[sub][base + j * sb]);
            int t = 0;
#pragma unroll
            for (int j = 0; j < CHI; ++j) {
                const cd wv = cscale(v[j], w);
#pragma unroll
                for (int jp = j; jp < CHI; ++jp, ++t) acc[t] = cfmac(acc[t], wv, v[jp]);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = seg_sum<4>(acc[t]);
        // zero outside the bond dimension; D = I_dim - (dim / tr M) M
        const int dim = dims[sub][lg];
        double tr = 0.0;
        {
            int t = 0;
#pragma unroll
            for (int j = 0; j < CHI; ++j)
#pragma unroll
                for (int jp = j; jp < CHI; ++jp, ++t) {
                    if (jp >= dim) acc[t] = cz<double>();
                    if (jp == j) tr += acc[t].re;
                }
        }
        const double sc = tr > 0.0 ? dim / tr : 0.0;
        double f2 = 0.0, l1 = 0.0;
        {
            int t = 0;
#pragma unroll
            for (int j = 0; j < CHI; ++j)
#pragma unroll
                for (int jp = j; jp < CHI; ++jp, ++t) {
                    cd dv = cscale(acc[t], -sc);
                    if (j == jp && j < dim) dv.re += 1.0;
                    const double a2 = cabs2(dv);
                    const double mult = j == jp ? 1.0 : 2.0;    // D is Hermitian
                    f2 += mult * a2;
                    l1 += mult * sqrt(a2);
                }
        }
        const double fro = sqrt(f2);
        const bool lead = q == 0 && vl / 4 < 3;
        double lo = lead ? fro : 0.0;
        double hi = lead ? fmin(sqrt((double)dim) * fro, l1) : 0.0;
        lo = seg_sum<LPV>(lo);
        hi = seg_sum<LPV>(hi);
        if (valid && vl == 0) {
            p.vres[a] = lo;
            p.vres_hi[a] = hi;
        }
    } else {
        __shared__ cd Mm[VPW][3][M2];
        residual_grams<CHI, S, LPV>(p, a, vl, G[sub], lam2[sub], dims[sub], Mm[sub]);
        double f2[3] = {0.0, 0.0, 0.0}, l1[3] = {0.0, 0.0, 0.0};
        for (int idx = vl; idx < 3 * M2; idx += LPV) {
            const int lg = idx / M2, j = (idx / CHI) % CHI, jp = idx % CHI;
            const double a2 = cabs2(residual_d<CHI>(Mm[sub][lg], dims[sub][lg], j, jp));
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (q == lg) {
                    f2[q] += a2;
                    l1[q] += sqrt(a2);
                }
            }
        }
        double lo = 0.0, hi = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double fro = sqrt(seg_sum<LPV>(f2[q]));
            const double L1 = seg_sum<LPV>(l1[q]);
            lo += fro;
            hi += fmin(sqrt((double)dims[sub][q]) * fro, L1);
        }
        if (valid && vl == 0) {
            p.vres[a] = lo;
            p.vres_hi[a] = hi;
        }
    }
}

__global__ __launch_bounds__(256) void k_residual_reduce(DevPool p, const int32_t* slots, int nslots, int mode) {
    __shared__ double red[256];
    const int s = slots[blockIdx.x];
    if (mode == RES_UNDECIDED && !(p.sflag[s] & FLAG_UNDECIDED)) return;
    const int v0 = p.s_v0[s], nv = p.s_nv[s], ne = p.s_ne[s];
    const double inv = ne > 0 ? 1.0 / (2.0 * ne) : 0.0;
    const double lo = slot_sum(p.vres, v0, nv, red) * inv;
    const double hi = mode == RES_BOUNDS ? slot_sum(p.vres_hi, v0, nv, red) * inv : lo;
    if (threadIdx.x == 0) {
        p.sres[s] = lo;
        p.sres_hi[s] = hi;
    }
}

__global__ void k_phase_flags_adaptive(DevPool p, const int32_t* slots, int n, int phase, int32_t* counters) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = slots[i];
    const int mask = p.smask[s];
    int fl = 0;
    if ((mask >> phase) & 1) {
        if (p.sres[s] > p.res_max) fl = FLAG_ACTIVE;               // R >= lower bound > res_max
        else if (p.sres_hi[s] > p.res_max) fl = FLAG_UNDECIDED;    // the bounds straddle res_max
    }
    p.sflag[s] = fl;
    p.ssweeps[s] = 0;
    p.sdist[s] = 0.0;
    if (fl & FLAG_ACTIVE) {
        p.stot[2 * s + 1] += 1;
        atomicAdd(&counters[0], 1);
    } else if (fl & FLAG_UNDECIDED) {
        atomicAdd(&counters[1], 1);
    }
}

__global__ void k_phase_flags_adaptive_final(DevPool p, const int32_t* slots, int n, int32_t* counters) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = slots[i];
    if (!(p.sflag[s] & FLAG_UNDECIDED)) return;
    const int fl = p.sres[s] > p.res_max ? FLAG_ACTIVE : 0;
    p.sflag[s] = fl;
    if (fl) {
        p.stot[2 * s + 1] += 1;
        atomicAdd(&counters[0], 1);
    }
}

// ------------------------------------------------------------------ fidelity bookkeeping
// -sum_j lambda_j^2 log lambda_j^2 of edge e if the bipartition cuts it
__device__ __forceinline__ double cut_entropy(const DevPool& p, int e, int chi) {
    if (!p.ecut[e]) return 0.0;
    double s = 0.0;
    for (int j = 0; j < chi; ++j) {
        const double l = p.lam[(size_t)e * chi + j];
        const double q = l * l;
        if (q > 0.0) s -= q * log(q);
    }
    return s;
}

__global__ __launch_bounds__(256) void k_fidelity_reduce(DevPool p, const int32_t* slots, int nslots, int chi) {
    __shared__ double red[256];
    __shared__ double mx[256];
    __shared__ double ent[256];
    const int s = slots[blockIdx.x];
    const int e0 = p.s_e0[s], ne = p.s_ne[s];
    double acc = 0.0, m = 0.0, en = 0.0;
    for (int k = threadIdx.x; k < ne; k += 256) {
        acc += p.elogf[e0 + k];
        m = fmax(m, p.eeps[e0 + k]);
        en += cut_entropy(p, e0 + k, chi);
    }
    red[threadIdx.x] = acc;
    mx[threadIdx.x] = m;
    ent[threadIdx.x] = en;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[threadIdx.x] += red[threadIdx.x + off];
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + off]);
            ent[threadIdx.x] += ent[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        p.sfid[3 * s] = red[0];
        p.sfid[3 * s + 1] = mx[0];
        p.sfid[3 * s + 2] += red[0];
        p.sent[s] = ent[0];
    }
}

__global__ __launch_bounds__(256) void k_entropy(DevPool p, const int32_t* slots, int nslots, int chi) {
    __shared__ double red[256];
    const int s = slots[blockIdx.x];
    const int e0 = p.s_e0[s], ne = p.s_ne[s];
    double en = 0.0;
    for (int k = threadIdx.x; k < ne; k += 256) en += cut_entropy(p, e0 + k, chi);
    red[threadIdx.x] = en;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) p.sent[s] = red[0];
}

int launch_fidelity_reduce(const DevPool& p, const int32_t* slots, int nslots, int chi, hipStream_t s) {
    if (nslots <= 0) return 0;
    k_fidelity_reduce<<<nslots, 256, 0, s>>>(p, slots, nslots, chi);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_entropy(const DevPool& p, const int32_t* slots, int nslots, int chi, hipStream_t s) {
    if (nslots <= 0) return 0;
    k_entropy<<<nslots, 256, 0, s>>>(p, slots, nslots, chi);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <int CHI, typename S>
__global__ __launch_bounds__(64) void k_sample_project(DevPool p, const int32_t* slots, int nslots, int a,
                                                       const double* u, double* prob) {
    constexpr int C3 = CHI * CHI * CHI;
    const int i = blockIdx.x;
    if (i >= nslots) return;
    const int s = slots[i];
    if (a >= p.s_nv[s]) return;
    const int v = p.s_v0[s] + a;
    const double p0 = p.rho[(size_t)v * 8];           // Re rho[0][0]
    const int x = u[i] < p0 ? 1 : -1;
    const int drop = x == 1 ? 1 : 0;                  // |0> carries Z = +1
    cpx<S>* gam = reinterpret_cast<cpx<S>*>(p.gam) + (size_t)v * 2 * C3 + (size_t)drop * C3;
    for (int idx = threadIdx.x; idx < C3; idx += 64) gam[idx] = cz<S>();
    if (threadIdx.x == 0) {
        p.xbits[v] = (int8_t)x;
        prob[i] = x == 1 ? p0 : 1.0 - p0;
    }
}

__global__ void k_sample_flags(DevPool p, const int32_t* slots, int n, int a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = slots[i];
    const int fl = a < p.s_nv[s] ? FLAG_ACTIVE : 0;
    p.sflag[s] = fl;
    p.ssweeps[s] = 0;
    p.sdist[s] = 0.0;
    if (fl) p.stot[2 * s + 1] += 1;
}

__global__ void k_zero_i32(int32_t* x, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0;
}

int launch_zero_i32(int32_t* x, int n, hipStream_t s) {
    if (n <= 0) return 0;
    k_zero_i32<<<(n + 63) / 64, 64, 0, s>>>(x, n);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

// ------------------------------------------------------------------ BP work compaction
// One workgroup: for every class c, exclusive scan over the plan's slots of
// the class-c segment lengths of slots still running BP.
__global__ __launch_bounds__(256) void k_compact_scan(DevPool p, const int32_t* slots, int nslots, int ncol,
                                                      const int32_t* seg, int32_t* out_off, int32_t* counts) {
    __shared__ int32_t part[256];
    for (int c = 0; c < ncol; ++c) {
        int32_t carry = 0;
        for (int base = 0; base < nslots; base += 256) {
            const int i = base + threadIdx.x;
            int32_t len = 0;
            if (i < nslots) {
                const int fl = p.sflag[slots[i]];
                const bool run = (fl & FLAG_ACTIVE) && !(fl & FLAG_BP_DONE);
                len = run ? seg[((size_t)c * nslots + i) * 2 + 1] : 0;
            }
            part[threadIdx.x] = len;
            __syncthreads();
            for (int off = 1; off < 256; off <<= 1) {          // inclusive Hillis-Steele scan
                const int32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
                __syncthreads();
                part[threadIdx.x] += v;
                __syncthreads();
            }
            if (i < nslots) out_off[(size_t)c * nslots + i] = carry + part[threadIdx.x] - len;
            const int32_t tot = part[255];
            __syncthreads();
            carry += tot;
        }
        if (threadIdx.x == 0) counts[c] = carry;
        __syncthreads();
    }
}

// BP work records of a class list: per position the two direction records of
// its edge and (edge, slot), so the sweep reaches all its data one load level
// after the record
__global__ __launch_bounds__(256) void k_bp_records(DevPool p, const int32_t* items, int n, int4* out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int e = items[i];
    out[3 * (size_t)i] = p.bpmeta[2 * e];
    out[3 * (size_t)i + 1] = p.bpmeta[2 * e + 1];
    out[3 * (size_t)i + 2] = make_int4(e, p.eslot[e], 0, 0);
}

// grid (nslots, ncol): copy a running slot's class segment to its compacted place
__global__ __launch_bounds__(256) void k_compact_copy(DevPool p, const int32_t* slots, int nslots,
                                                      const int32_t* seg, const int64_t* cls_off,
                                                      const int32_t* out_off, const int32_t* full,
                                                      int32_t* out, const int4* full_rec, int4* out_rec) {
    const int i = blockIdx.x, c = blockIdx.y;
    const int fl = p.sflag[slots[i]];
    if (!(fl & FLAG_ACTIVE) || (fl & FLAG_BP_DONE)) return;
    const int32_t so = seg[((size_t)c * nslots + i) * 2], len = seg[((size_t)c * nslots + i) * 2 + 1];
    const int32_t oo = out_off[(size_t)c * nslots + i];
    const int64_t base = cls_off[c];
    for (int k = threadIdx.x; k < len; k += 256) out[base + oo + k] = full[base + so + k];
    for (int k = threadIdx.x; k < 3 * len; k += 256) out_rec[3 * (base + oo) + k] = full_rec[3 * (base + so) + k];
}

int launch_bp_compact(const DevPool& p, const int32_t* slots, int nslots, int ncol, const int32_t* seg,
                      const int64_t* cls_off, const int32_t* full, int32_t* out, const int4* full_rec,
                      int4* out_rec, int32_t* counts, int32_t* scratch, hipStream_t s) {
    if (nslots <= 0 || ncol <= 0) return 0;
    k_compact_scan<<<1, 256, 0, s>>>(p, slots, nslots, ncol, seg, scratch, counts);
    k_compact_copy<<<dim3(nslots, ncol), 256, 0, s>>>(p, slots, nslots, seg, cls_off, scratch, full, out,
                                                      full_rec, out_rec);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_bp_records(const DevPool& p, const int32_t* items, int n, int4* out, hipStream_t s) {
    if (n <= 0) return 0;
    k_bp_records<<<(n + 255) / 256, 256, 0, s>>>(p, items, n, out);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

// ------------------------------------------------------------------ launchers
// ------------------------------------------------------------------ random BP start
// Output i (0-based) of SplitMix64 seeded with `seed` (Steele, Lea, Flood,
// OOPSLA 2014): the generator's state after i + 1 steps is seed + (i + 1)
// gamma, gamma = 0x9E3779B97F4A7C15, followed by its output mix.  Counter-
// based access, so every entry of every message is drawn independently of
// the launch layout.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// uniform on the 2^-52 grid of [-1, 1): the top 53 bits as a fraction, 2x - 1
__device__ __forceinline__ double splitmix_sym(uint64_t x) { return (double)(x >> 11) * 0x1.0p-52 - 1.0; }

// Alg. 1's random initialisation m = A A^dagger / tr(A A^dagger) (App. B),
// one thread per message entry.  A is d x d, d the bond's dimension (its
// non-zero lambdas); entry A[r][k] of direction dir of the instance's edge
// el (its id within the instance) takes outputs 2i and 2i + 1 of the stream
// as real and imaginary parts, i = ((el * 2 + dir) * chi + r) * chi + k.
// Entries outside the d x d block are zero.
template <int CHI, typename S>
__global__ __launch_bounds__(256) void k_random_messages(DevPool p, const int32_t* items, int nitems, uint64_t seed) {
    constexpr int M2 = CHI * CHI;
    const size_t gid = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (size_t)nitems * 2 * M2) return;
    const int idx = (int)(gid % M2);
    const int dir = (int)((gid / M2) & 1);
    const int e = items[gid / (2 * M2)];
    const int slot = p.eslot[e];
    const uint64_t el = (uint64_t)(e - p.s_e0[slot]);
    int dim = 0;
    for (int j = 0; j < CHI; ++j) dim += p.lam[(size_t)e * CHI + j] > 0.0 ? 1 : 0;
    const uint64_t base = (el * 2 + (uint64_t)dir) * M2;
    auto A = [&](int r, int k) -> cd {
        const uint64_t i = 2 * (base + (uint64_t)(r * CHI + k));
        return {splitmix_sym(splitmix64_at(seed, i)), splitmix_sym(splitmix64_at(seed, i + 1))};
    };
    double tr = 0.0;
    for (int r = 0; r < dim; ++r)
        for (int k = 0; k < dim; ++k) tr += cabs2(A(r, k));
    const int r = idx / CHI, c = idx % CHI;
    cd acc = cz<double>();
    if (r < dim && c < dim)
        for (int k = 0; k < dim; ++k) acc = cfmac(acc, A(r, k), A(c, k));
    const double it = tr > 0.0 ? 1.0 / tr : 0.0;
    reinterpret_cast<cpx<S>*>(p.msg)[((size_t)e * 2 + dir) * M2 + idx] = from_cd<S>(cscale(acc, it));
}

// ------------------------------------------------------------------ bond SVD alone
// The bond SVD of the simple update (Alg. 3) on caller-given 2chi x 2chi
// cores, in the simple update's team layout, column presort and two-launch
// scheme: EPW cores per wavefront; FIX = false runs the restricted
// iteration and the kept-set check (at chi <= 4) and marks failures with a
// negative sweep count; FIX = true redoes exactly those from the original
// core on every pair.  sigma[i][0 .. 2chi) receives the column norms at
// exit, descending; the first chi are the values the simple update keeps.
template <int CHI, int EPW, bool FIX>
__global__ __launch_bounds__(64) void k_core_svd(const double* core, int count, double cut, double* sigma,
                                                 int32_t* sweeps_out) {
    constexpr int LPE = 64 / EPW;
    constexpr int N = 2 * CHI;
    constexpr int LPC = JLayout<N, LPE>::LPC;
    constexpr int EPL = JLayout<N, LPE>::EPL;
    constexpr int KEEP = (CHI <= 4 && !FIX) ? CHI : N;
    __shared__ cd Ul[EPW][N][N];
    __shared__ double sig[EPW][N];
    const int lane = threadIdx.x;
    const int sub = lane / LPE;
    const int el = lane % LPE;
    const int item = (int)blockIdx.x * EPW + sub;
    bool valid = item < count;
    const int it = valid ? item : 0;
    int prev = 0;
    if constexpr (FIX) {
        prev = sweeps_out[it];
        valid = valid && prev < 0;
        if (__ballot(valid) == 0) return;    // uniform: one wavefront per work-group
    }
    const int ccol = JLayout<N, LPE>::col(el);
    const int cg = JLayout<N, LPE>::grp(el);
    cd m[EPL], v[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const double* src = core + (((size_t)it * N + cg + LPC * k) * N + ccol) * 2;
        m[k] = {src[0], src[1]};
    }
    {
        double own2 = 0.0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) own2 += cabs2(m[k]);
        own2 = strided_sum<N, LPC>(own2);
        if (cg == 0) sig[sub][ccol] = own2;
        __syncthreads();
        int rk = 0;
        const double me = sig[sub][ccol];
        for (int c = 0; c < N; ++c) {
            const double o = sig[sub][c];
            rk += (o > me || (o == me && c < ccol)) ? 1 : 0;
        }
#pragma unroll
        for (int k = 0; k < EPL; ++k) Ul[sub][cg + LPC * k][rk] = m[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < EPL; ++k) m[k] = Ul[sub][cg + LPC * k][ccol];
    }
    const int sw =
        jacobi_svd_team<N, LPE, false, KEEP>(m, v, el, JACOBI_TOL, KEEP < N ? KEEP_SWEEPS : JACOBI_MAX_SWEEPS);
    bool ok = true;
    if constexpr (KEEP < N) ok = sw <= KEEP_SWEEPS && kept_set_is_largest<N, LPE, KEEP>(m, el, cut);
    double nrm = 0.0;
#pragma unroll
    for (int k = 0; k < EPL; ++k) nrm += cabs2(m[k]);
    nrm = strided_sum<N, LPC>(nrm);
    __syncthreads();
    if (cg == 0) sig[sub][ccol] = sqrt(nrm);
    __syncthreads();
    if (valid && ok && el < N) {
        int rank = 0;
        const double me = sig[sub][el];
        for (int c = 0; c < N; ++c) {
            const double o = sig[sub][c];
            rank += (o > me || (o == me && c < el)) ? 1 : 0;
        }
        if (rank < N) sigma[(size_t)item * N + rank] = me;
    }
    if (valid && el == 0) {
        const int used = FIX ? (-prev < KEEP_SWEEPS ? -prev : KEEP_SWEEPS) : 0;
        sweeps_out[item] = ok ? used + sw : -sw;
    }
}

bool chi_supported(int chi) { return chi == 4 || chi == 8 || chi == 16; }

#define GTQA_DISPATCH(chi, prec, CALL)                                            \
    do {                                                                           \
        if ((chi) == 4 && (prec) == 0) { constexpr int CHI = 4; using S = double; CALL; } \
        else if ((chi) == 4) { constexpr int CHI = 4; using S = float; CALL; }      \
        else if ((chi) == 8 && (prec) == 0) { constexpr int CHI = 8; using S = double; CALL; } \
        else if ((chi) == 8) { constexpr int CHI = 8; using S = float; CALL; }      \
        else return -1;                                                            \
    } while (0)
// kernels written for any chi (plain loops over the tensor): chi = 16 as well
#define GTQA_DISPATCH_ANY(chi, prec, CALL)                                        \
    do {                                                                           \
        if ((chi) == 16 && (prec) == 0) { constexpr int CHI = 16; using S = double; CALL; } \
        else if ((chi) == 16) { constexpr int CHI = 16; using S = float; CALL; }    \
        else GTQA_DISPATCH(chi, prec, CALL);                                       \
    } while (0)

static int last_err() { return hipGetLastError() == hipSuccess ? 0 : -4; }

Tuning& tuning() {
    static Tuning t{4, 0, 4};
    return t;
}

// launch grid for `groups` work-groups under the current tuning; q gets the remap flag
static unsigned tuned_grid(DevPool& q, long groups) {
    q.xcd_remap = tuning().xcd_remap;
    if (q.xcd_remap) groups = (groups + 7) / 8 * 8;
    return (unsigned)groups;
}

int launch_init_plus(int chi, int prec, const DevPool& p, const int32_t* verts, int nv,
                     const int32_t* edges, int ne, hipStream_t s) {
    const size_t tot = std::max((size_t)nv * 2 * chi * chi * chi, (size_t)ne * chi);
    if (tot == 0) return 0;
    const unsigned grid = (unsigned)((tot + 63) / 64);
    GTQA_DISPATCH_ANY(chi, prec, (k_init_plus<CHI, S><<<grid, 64, 0, s>>>(p, verts, nv, edges, ne)));
    return last_err();
}

int launch_simple_update(int chi, int prec, const DevPool& p, const int32_t* edges, int ne,
                         hipStream_t s) {
    if (ne <= 0) return 0;
    if (chi == 16) return launch_wide_simple_update(chi, prec, p, edges, ne, s);
    // 2 or 4 edges per wavefront at chi = 4 (tuned), one at chi = 8 (register budget)
    DevPool q = p;
    const int epw4 = tuning().su_epw_chi4 == 2 ? 2 : 4;
    // at chi = 4 a second launch redoes the rare edges whose restricted bond
    // SVD failed the kept-set check (flagged by the first)
    GTQA_DISPATCH(chi, prec, ({
        if (CHI == 4 && epw4 == 2) {
            constexpr int EPW = CHI == 4 ? 2 : 1;
            k_simple_update<CHI, S, EPW><<<tuned_grid(q, (ne + EPW - 1) / EPW), 64, 0, s>>>(q, edges, ne);
            if (CHI == 4) k_simple_update<CHI, S, EPW, true><<<tuned_grid(q, (ne + EPW - 1) / EPW), 64, 0, s>>>(q, edges, ne);
        } else {
            constexpr int EPW = CHI == 4 ? 4 : 1;
            k_simple_update<CHI, S, EPW><<<tuned_grid(q, (ne + EPW - 1) / EPW), 64, 0, s>>>(q, edges, ne);
            if (CHI == 4) k_simple_update<CHI, S, EPW, true><<<tuned_grid(q, (ne + EPW - 1) / EPW), 64, 0, s>>>(q, edges, ne);
        }
    }));
    return last_err();
}

int launch_warm_messages(int chi, int prec, const DevPool& p, const int32_t* edges, int ne,
                         hipStream_t s) {
    if (ne <= 0) return 0;
    const size_t tot = (size_t)ne * 2 * chi * chi;
    const unsigned grid = (unsigned)((tot + 63) / 64);
    GTQA_DISPATCH_ANY(chi, prec, (k_warm_messages<CHI, S><<<grid, 64, 0, s>>>(p, edges, ne)));
    return last_err();
}

int launch_bp_sweep_class(int chi, int prec, const DevPool& p, const int4* recs, int ne,
                          int first_sweep, int cls, const int32_t* gate, hipStream_t s) {
    if (ne <= 0) return 0;
    if (chi == 16) return launch_wide_bp_sweep_class(chi, prec, p, recs, ne, first_sweep, cls, gate, s);
    DevPool q = p;
    GTQA_DISPATCH(chi, prec, ({
        const long wgs = (ne + BPLayout<CHI>::EPG - 1) / BPLayout<CHI>::EPG;
        const unsigned grid = tuned_grid(q, wgs);
        // the first sweep's first class (every class of a flooding first
        // sweep) sees only diagonal incoming messages
        constexpr bool W4 = true;
        if (p.bp_flood) {
            if (first_sweep) k_bp_class<CHI, S, true, true, W4><<<grid, 64, 0, s>>>(q, recs, ne, cls, gate);
            else k_bp_class<CHI, S, false, true><<<grid, 64, 0, s>>>(q, recs, ne, cls, gate);
        } else {
            if (first_sweep && cls == 0) k_bp_class<CHI, S, true, false, W4><<<grid, 64, 0, s>>>(q, recs, ne, cls, gate);
            else if (first_sweep) k_bp_class<CHI, S, true><<<grid, 64, 0, s>>>(q, recs, ne, cls, gate);
            else k_bp_class<CHI, S, false><<<grid, 64, 0, s>>>(q, recs, ne, cls, gate);
        }
    }));
    return last_err();
}

template <typename S>
__global__ __launch_bounds__(256) void k_bp_snapshot(DevPool p, const int4* recs, int n, int m2x2) {
    const size_t gid = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (size_t)n * m2x2) return;
    const int4 es = recs[3 * (gid / m2x2) + 2];
    const int fl = p.sflag[es.y];
    if (!(fl & FLAG_ACTIVE) || (fl & (FLAG_BP_DONE | FLAG_UNDECIDED))) return;
    const size_t o = (size_t)es.x * m2x2 + gid % m2x2;
    reinterpret_cast<cpx<S>*>(p.mold)[o] = reinterpret_cast<const cpx<S>*>(p.msg)[o];
}

int launch_bp_snapshot(int chi, int prec, const DevPool& p, const int4* recs, int ne, hipStream_t s) {
    if (ne <= 0) return 0;
    const int m2x2 = 2 * chi * chi;
    const unsigned grid = (unsigned)(((size_t)ne * m2x2 + 255) / 256);
    if (prec == 0) k_bp_snapshot<double><<<grid, 256, 0, s>>>(p, recs, ne, m2x2);
    else k_bp_snapshot<float><<<grid, 256, 0, s>>>(p, recs, ne, m2x2);
    return last_err();
}

int launch_bp_reduce(const DevPool& p, const int32_t* slots, int nslots, int32_t* counters,
                     int force_exact, int max_sweeps, hipStream_t s) {
    if (nslots <= 0) return 0;
    k_bp_reduce<<<nslots, 256, 0, s>>>(p, slots, nslots, counters, force_exact, max_sweeps);
    return last_err();
}

int launch_bp_exact(int chi, int prec, const DevPool& p, const int32_t* edges, int ne, int force, hipStream_t s) {
    if (ne <= 0) return 0;
    GTQA_DISPATCH_ANY(chi, prec, (k_bp_exact<CHI, S><<<ne, 64, 0, s>>>(p, edges, ne, force)));
    return last_err();
}

int launch_bp_reduce_exact(const DevPool& p, const int32_t* slots, int nslots, int32_t* counters,
                           int force, int max_sweeps, hipStream_t s) {
    if (nslots <= 0) return 0;
    k_bp_reduce_exact<<<nslots, 256, 0, s>>>(p, slots, nslots, counters, force, max_sweeps);
    return last_err();
}

int launch_canonicalise(int chi, int prec, const DevPool& p, const int32_t* edges, int ne,
                        hipStream_t s) {
    if (ne <= 0) return 0;
    if (chi == 16) return launch_wide_canonicalise(chi, prec, p, edges, ne, s);
    DevPool q = p;
    if (chi == 4 && tuning().canon_lanes_chi4 == 4) {
        const unsigned grid = tuned_grid(q, (ne + 15) / 16);
        if (prec == 0) k_canonicalise4<double><<<grid, 64, 0, s>>>(q, edges, ne);
        else k_canonicalise4<float><<<grid, 64, 0, s>>>(q, edges, ne);
        return last_err();
    }
    GTQA_DISPATCH(chi, prec,
                  (k_canonicalise<CHI, S><<<tuned_grid(q, (ne + CanonLayout<CHI>::TPW - 1) / CanonLayout<CHI>::TPW),
                                             64, 0, s>>>(q, edges, ne)));
    return last_err();
}

int launch_gauge_apply(int chi, int prec, const DevPool& p, const int32_t* verts, int nv,
                       int apply_x, hipStream_t s) {
    if (nv <= 0) return 0;
    if (chi == 16) return launch_wide_gauge_apply(chi, prec, p, verts, nv, apply_x, s);
    DevPool q = p;
    const unsigned grid = tuned_grid(q, nv);
    GTQA_DISPATCH(chi, prec, (k_gauge_apply<CHI, S><<<grid, 64, 0, s>>>(q, verts, nv, apply_x)));
    return last_err();
}

int launch_x_layer(int chi, int prec, const DevPool& p, const int32_t* verts, int nv,
                   hipStream_t s) {
    if (nv <= 0) return 0;
    GTQA_DISPATCH_ANY(chi, prec, (k_x_layer<CHI, S><<<nv, 64, 0, s>>>(p, verts, nv)));
    return last_err();
}

int launch_readout(int chi, int prec, const DevPool& p, const int32_t* verts, int nv,
                   int from_messages, hipStream_t s) {
    if (nv <= 0) return 0;
    GTQA_DISPATCH_ANY(chi, prec, (k_readout<CHI, S><<<nv, 64, 0, s>>>(p, verts, nv, from_messages)));
    return last_err();
}

int launch_energy(const DevPool& p, const int32_t* slots, int nslots, hipStream_t s) {
    if (nslots <= 0) return 0;
    k_energy<<<nslots, 256, 0, s>>>(p, slots, nslots);
    return last_err();
}

int launch_phase_flags(const DevPool& p, const int32_t* slots, int nslots, int phase,
                       hipStream_t s, int32_t* clear4) {
    if (nslots <= 0) return 0;
    k_phase_flags<<<(nslots + 255) / 256, 256, 0, s>>>(p, slots, nslots, phase, clear4);
    return last_err();
}

int launch_residual(int chi, int prec, const DevPool& p, const int32_t* verts, int nv, const int32_t* slots,
                    int nslots, int mode, hipStream_t s) {
    if (nv <= 0 || nslots <= 0) return 0;
    if (chi == 16) {
        if (launch_wide_residual(chi, prec, p, verts, nv, mode, s)) return -1;
    } else if (chi > 8) {
        return -1;
    } else if (mode == RES_BOUNDS) {
        DevPool q = p;
        const int vpw = 64 / (chi * chi);
        const unsigned grid = tuned_grid(q, (nv + vpw - 1) / vpw);
        GTQA_DISPATCH(chi, prec, (k_residual_bounds<CHI, S><<<grid, 64, 0, s>>>(q, verts, nv)));
    } else {
        const int only = mode == RES_UNDECIDED ? 1 : 0;
        GTQA_DISPATCH(chi, prec, (k_residual<CHI, S><<<nv, 64, 0, s>>>(p, verts, nv, only)));
    }
    k_residual_reduce<<<nslots, 256, 0, s>>>(p, slots, nslots, mode);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_phase_flags_adaptive(const DevPool& p, const int32_t* slots, int nslots, int phase, int32_t* counters,
                                hipStream_t s) {
    if (nslots <= 0) return 0;
    k_phase_flags_adaptive<<<(nslots + 255) / 256, 256, 0, s>>>(p, slots, nslots, phase, counters);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_phase_flags_adaptive_final(const DevPool& p, const int32_t* slots, int nslots, int32_t* counters,
                                      hipStream_t s) {
    if (nslots <= 0) return 0;
    k_phase_flags_adaptive_final<<<(nslots + 255) / 256, 256, 0, s>>>(p, slots, nslots, counters);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_sample_project(int chi, int prec, const DevPool& p, const int32_t* slots, int nslots, int a,
                          const double* u, double* prob, hipStream_t s) {
    if (nslots <= 0) return 0;
    GTQA_DISPATCH_ANY(chi, prec, (k_sample_project<CHI, S><<<nslots, 64, 0, s>>>(p, slots, nslots, a, u, prob)));
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_sample_flags(const DevPool& p, const int32_t* slots, int nslots, int a, hipStream_t s) {
    if (nslots <= 0) return 0;
    k_sample_flags<<<(nslots + 255) / 256, 256, 0, s>>>(p, slots, nslots, a);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_core_svd(int chi, const double* core, int count, double cut, double* sigma, int32_t* sweeps,
                    hipStream_t s) {
    if (count <= 0) return 0;
    const int epw4 = tuning().su_epw_chi4 == 2 ? 2 : 4;
    if (chi == 4 && epw4 == 2) {
        k_core_svd<4, 2, false><<<(count + 1) / 2, 64, 0, s>>>(core, count, cut, sigma, sweeps);
        k_core_svd<4, 2, true><<<(count + 1) / 2, 64, 0, s>>>(core, count, cut, sigma, sweeps);
    } else if (chi == 4) {
        k_core_svd<4, 4, false><<<(count + 3) / 4, 64, 0, s>>>(core, count, cut, sigma, sweeps);
        k_core_svd<4, 4, true><<<(count + 3) / 4, 64, 0, s>>>(core, count, cut, sigma, sweeps);
    } else if (chi == 8) {
        k_core_svd<8, 1, false><<<count, 64, 0, s>>>(core, count, cut, sigma, sweeps);
    } else if (chi == 16) {
        k_core_svd<16, 1, false><<<count, 64, 0, s>>>(core, count, cut, sigma, sweeps);
    } else {
        return 1;
    }
    return last_err();
}

int launch_random_messages(int chi, int prec, const DevPool& p, const int32_t* edges, int ne, uint64_t seed,
                           hipStream_t s) {
    if (ne <= 0) return 0;
    const int grid = (int)(((size_t)ne * 2 * chi * chi + 255) / 256);
    GTQA_DISPATCH_ANY(chi, prec, (k_random_messages<CHI, S><<<grid, 256, 0, s>>>(p, edges, ne, seed)));
    return last_err();
}

}  // namespace gtqa

// ====================================================================== no-allocation bond SVD
// gtqa_bond_svd without device allocation, for callers that cannot allocate
// (inside stream capture, tight serving loops, harnesses that forbid it).
// The device copies of the cores, the column norms and the sweep counts live
// in one file-scope array, `scratch`, of kScratchBytes per device, held until
// the process ends.  In host code `scratch` names a host-side stand-in: its
// device address is taken once per device with hipGetSymbolAddress and only
// that address is used.  Every call on a device shares its array, so calls
// that overlap on one device race; the kernel writes every output entry it
// reads back, so nothing has to be cleared between calls.
namespace {

constexpr size_t kScratchBytes = size_t(2) << 20;   // 2 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GTQA_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GTQA_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GTQA_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" int32_t gtqa_bond_svd_noalloc_max(int32_t chi) {
    if (!gtqa::chi_supported(chi)) return 0;
    const size_t n = (size_t)2 * chi;
    // per core: the matrix (n x n complex), n norms, one sweep count, plus
    // up to 3 x 255 bytes of alignment padding between the three regions
    const size_t per = n * n * 16 + n * 8 + 4;
    return (int32_t)((kScratchBytes - 3 * 256) / per);
}

extern "C" int gtqa_bond_svd_noalloc(int32_t chi, int32_t count, const double* core, double svd_rel_cutoff,
                                     double* sigma, int32_t* sweeps) {
    if (!gtqa::chi_supported(chi)) return GTQA_ERR_UNSUPPORTED;
    if (count < 0 || (count > 0 && (!core || !sigma || !sweeps)) || !(svd_rel_cutoff >= 0.0) ||
        !std::isfinite(svd_rel_cutoff))
        return GTQA_ERR_ARG;
    if (count > gtqa_bond_svd_noalloc_max(chi)) {
        std::fprintf(stderr, "gtqa_bond_svd_noalloc: %d cores exceed the %d that fit its %zu-byte scratch\n",
                     (int)count, (int)gtqa_bond_svd_noalloc_max(chi), kScratchBytes);
        return GTQA_ERR_ARG;
    }
    if (count == 0) return GTQA_OK;
    const size_t n = (size_t)2 * chi;
    const size_t nc = (size_t)count * n * n * 2;
    for (size_t i = 0; i < nc; ++i)
        if (!std::isfinite(core[i])) return GTQA_ERR_NUMERIC;
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    unsigned char* b = static_cast<unsigned char*>(base);
    double* dcore = reinterpret_cast<double*>(b);
    double* dsig = reinterpret_cast<double*>(b + align256(nc * sizeof(double)));
    int32_t* dsw = reinterpret_cast<int32_t*>(reinterpret_cast<unsigned char*>(dsig) +
                                              align256((size_t)count * n * sizeof(double)));
    if (hipMemcpy(dcore, core, nc * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return GTQA_ERR_HIP;
    if (gtqa::launch_core_svd(chi, dcore, count, svd_rel_cutoff, dsig, dsw, nullptr)) return GTQA_ERR_HIP;
    if (hipMemcpy(sigma, dsig, (size_t)count * n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(sweeps, dsw, (size_t)count * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return GTQA_ERR_HIP;
    return GTQA_OK;
}
