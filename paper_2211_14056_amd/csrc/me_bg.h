// Table-driven colour-ordered recursion: one wavefront per event.
//
// The straight-line kernels keep a whole event in one lane; their code and working
// set grow with the number of diagrams, which is where the paper finds generic code
// degrading (sect. 2, the discussion of Table 1; sect. 3, Fig. 4).  For
// g g -> t tbar g g g (120 colour orderings, 165 currents, 206 quark-line prefixes per
// helicity) the event is spread over the 64 lanes of a wavefront instead: the nodes of
// one level of the recursion are independent, so the lanes take the currents of one
// length, then the quark-line prefixes of one length, then the orderings, then the rows
// of the colour matrix.  The tables (gen/bg_tables.py) hold the splits; the vertex
// forms, the quark line and the colour matrix are those of the straight-line code
// (gen/process_compiler.py), so the same table kernel for 3 and 4 gluons reproduces the
// straight-line kernels.  Currents, prefixes and amplitudes live in LDS (11.7 KB per event
// in FP32, 23 KB in FP64), kinematics are evaluated once per event in FP64 and rounded.
#pragma once
#include "internal.h"
#include "me_common.h"

namespace mf {

// BgTab<K>: the generated tables of the K-gluon recursion (generated/me_bg_k<K>.inc)
template <int K> struct BgTab;

template <int K, typename R>
struct BgShared {
    static constexpr int NCUR = BgTab<K>::NCUR, NPRE = BgTab<K>::NPRE_STORED, NORD = BgTab<K>::NORD;
    R J[NCUR][8];             // currents, light-cone components (+, -, t, tb) x (re, im)
    R Q[NPRE][8];             // quark-line row spinors after the prefixes shorter than K - 1,
                              // propagator included
    R A[2][NORD][2];          // amplitudes per antitop helicity
    R P[1 << K][4];           // gluon-subset momentum sums (incoming convention): E+z, E-z, x, y
    R ig[1 << K];             // 1 / P^2
    R qp[1 << K][5];          // (q+, q-, qx, qy, m_t) / (q^2 - m_t^2), q = p_t - P
    R eu[K][5];               // outgoing gluons' polarisation basis / sqrt 2: u (x, y, z), w (x, y)
    R ub[2][8], vs[2][8];     // top and antitop spinors for both helicities
    double pe[K + 2][4];      // the event's momenta (FP64), read by index from every lane
};

template <typename R>
struct cx {
    R re, im;
};
template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b)
{
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
template <typename R> __device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c)
{
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
template <typename R> __device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return {a.re * s, a.im * s}; }

template <typename R>
struct V4c {
    cx<R> c[4];
};

template <typename R> __device__ __forceinline__ V4c<R> load8(const R* v, R sgn)
{
    V4c<R> r;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) r.c[mu] = {sgn * v[2 * mu], sgn * v[2 * mu + 1]};
    return r;
}
template <typename R> __device__ __forceinline__ void store8(R* v, const V4c<R>& x)
{
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        v[2 * mu] = x.c[mu].re;
        v[2 * mu + 1] = x.c[mu].im;
    }
}

// 2 x.y in light-cone components: x+ y- + x- y+ - xt ytb - xtb yt
template <typename R> __device__ __forceinline__ cx<R> dot2(const V4c<R>& x, const V4c<R>& y)
{
    cx<R> r = cmul(x.c[0], y.c[1]);
    r = cfma(x.c[1], y.c[0], r);
    r = cfma({-x.c[2].re, -x.c[2].im}, y.c[3], r);
    r = cfma({-x.c[3].re, -x.c[3].im}, y.c[2], r);
    return r;
}

// real momentum (E+z, E-z, x, y) as a light-cone complex vector
template <typename R> __device__ __forceinline__ V4c<R> mom_lc(const R* P)
{
    return V4c<R>{{{P[0], R(0)}, {P[1], R(0)}, {P[2], P[3]}, {P[2], -P[3]}}};
}

// row spinor psi times Jslash (light cone): one term per spinor component, added to out
template <typename R> __device__ __forceinline__ void slash_row_add(const V4c<R>& psi, const V4c<R>& J, V4c<R>& out)
{
    out.c[0] = cfma(psi.c[3], J.c[2], cfma(psi.c[2], J.c[0], out.c[0]));
    out.c[1] = cfma(psi.c[3], J.c[1], cfma(psi.c[2], J.c[3], out.c[1]));
    out.c[2] = cfma({-psi.c[1].re, -psi.c[1].im}, J.c[2], cfma(psi.c[0], J.c[1], out.c[2]));
    out.c[3] = cfma(psi.c[1], J.c[0], cfma({-psi.c[0].re, -psi.c[0].im}, J.c[3], out.c[3]));
}

template <int K>
constexpr double bg_norm_noalpha()
{
    // 2 (reversed helicities) / (initial average 256 * identical final gluons * colour denominator)
    double sym = 1.0;
    for (int i = 2; i <= K - 2; ++i) sym *= i;
    return 2.0 / (256.0 * sym * BgTab<K>::CDEN);
}

// |M|^2 of one event without couplings and normalisation, computed by the LPE lanes of the
// calling group (lane = this lane's index in the group; every lane of the workgroup must
// call it, since it synchronises the workgroup between levels); returned in every lane of
// the group.
template <int K, typename R, int LPE>
__device__ double bg_event(const double (&pe)[K + 2][4], double mt, BgShared<K, R>& sh, int lane)
{
    typedef BgTab<K> T;
    constexpr int NS = 1 << K;
    // ---- kinematics (FP64, rounded): incoming-convention gluon momenta k_g
    // gluon g is leg g for g < 2 (incoming) and leg g + 2 otherwise (outgoing)
    auto kcomp = [&](int g, int c) { return g < 2 ? pe[g][c] : -pe[g + 2][c]; };
    for (int m = lane; m < NS; m += LPE) {
        double P[4] = {0.0, 0.0, 0.0, 0.0};
        int cnt = 0;
        for (int g = 0; g < K; ++g)
            if (m >> g & 1) {
                ++cnt;
#pragma unroll
                for (int c = 0; c < 4; ++c) P[c] += kcomp(g, c);
            }
        sh.P[m][0] = R(P[0] + P[3]);
        sh.P[m][1] = R(P[0] - P[3]);
        sh.P[m][2] = R(P[1]);
        sh.P[m][3] = R(P[2]);
        sh.ig[m] = cnt >= 2 ? R(1.0 / (P[0] * P[0] - P[1] * P[1] - P[2] * P[2] - P[3] * P[3])) : R(0);
        if (cnt >= 1 && cnt < K) {
            double q[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) q[c] = pe[2][c] - P[c];
            const double iq = 1.0 / ((q[0] - q[3]) * (q[0] + q[3]) - q[1] * q[1] - q[2] * q[2] - mt * mt);
            sh.qp[m][0] = R((q[0] + q[3]) * iq);
            sh.qp[m][1] = R((q[0] - q[3]) * iq);
            sh.qp[m][2] = R(q[1] * iq);
            sh.qp[m][3] = R(q[2] * iq);
            sh.qp[m][4] = R(mt * iq);
        }
    }
    for (int g = 2 + lane; g < K; g += LPE) {
        R u[3], w[2];
        pol_basis<R, double>(pe[g + 2], u, w);
        sh.eu[g][0] = u[0]; sh.eu[g][1] = u[1]; sh.eu[g][2] = u[2];
        sh.eu[g][3] = w[0]; sh.eu[g][4] = w[1];
    }
    if (lane == LPE - 1) {
        cplx<R> s[4];
        for (int h = 0; h < 2; ++h) {
            ubar_spinor<R, double>(pe[2], mt, h ? 1 : -1, s);
            for (int j = 0; j < 4; ++j) { sh.ub[h][2 * j] = s[j].re; sh.ub[h][2 * j + 1] = s[j].im; }
            v_spinor<R, double>(pe[3], mt, h ? 1 : -1, s);
            for (int j = 0; j < 4; ++j) { sh.vs[h][2 * j] = s[j].re; sh.vs[h][2 * j + 1] = s[j].im; }
        }
    }
    __syncthreads();
    const R r2 = R(0.70710678118654752440);
    R acc = R(0);
#pragma unroll 1
    for (int gconf = 1 << (K - 1); gconf < (1 << K); ++gconf) {     // last gluon: helicity +1
        // ---- external currents
        for (int g = lane; g < K; g += LPE) {
            const R l = (gconf >> g) & 1 ? R(1) : R(-1);
            V4c<R> e;
            if (g == 0) {
                e = V4c<R>{{{R(0), R(0)}, {R(0), R(0)}, {(R(1) - l) * r2, R(0)}, {-(R(1) + l) * r2, R(0)}}};
            } else if (g == 1) {
                e = V4c<R>{{{R(0), R(0)}, {R(0), R(0)}, {(R(1) + l) * r2, R(0)}, {(l - R(1)) * r2, R(0)}}};
            } else {
                const R* b = sh.eu[g];
                const R ez = -l * b[2];
                e = V4c<R>{{{ez, R(0)}, {-ez, R(0)}, {fma(-l, b[0], -b[4]), fma(-l, b[1], b[3])},
                            {fma(-l, b[0], b[4]), fma(l, b[1], b[3])}}};
            }
            store8(sh.J[g], e);
        }
        __syncthreads();
        // ---- multi-gluon currents, by length
#pragma unroll 1
        for (int L = 2; L <= K; ++L) {
            for (int c = T::cur_levels(L - 1) + lane; c < T::cur_levels(L); c += LPE) {
                V4c<R> t{};
                const int n3 = T::cur_n3(c), n4 = T::cur_n4(c);
                for (int s = 0; s < n3; ++s) {
                    const short* sp = T::cur_s3(c, s);
                    const V4c<R> Ja = load8(sh.J[sp[0]], (sp[4] & 1) ? R(-1) : R(1));
                    const V4c<R> Jb = load8(sh.J[sp[1]], (sp[4] & 2) ? R(-1) : R(1));
                    const V4c<R> Pa = mom_lc(sh.P[sp[2]]), Pb = mom_lc(sh.P[sp[3]]);
                    const cx<R> dab = dot2(Ja, Jb);
                    const cx<R> hd = {dab.re * R(0.5), dab.im * R(0.5)};
                    const cx<R> pbja = dot2(Pb, Ja), pajb = dot2(Pa, Jb);
#pragma unroll
                    for (int mu = 0; mu < 4; ++mu) {
                        const cx<R> dP = {Pa.c[mu].re - Pb.c[mu].re, Pa.c[mu].im - Pb.c[mu].im};
                        t.c[mu] = cfma(hd, dP, t.c[mu]);
                        t.c[mu] = cfma(pbja, Jb.c[mu], t.c[mu]);
                        t.c[mu] = cfma({-pajb.re, -pajb.im}, Ja.c[mu], t.c[mu]);
                    }
                }
                for (int s = 0; s < n4; ++s) {
                    const short* sp = T::cur_s4(c, s);
                    const V4c<R> Ja = load8(sh.J[sp[0]], (sp[3] & 1) ? R(-1) : R(1));
                    const V4c<R> Jb = load8(sh.J[sp[1]], (sp[3] & 2) ? R(-1) : R(1));
                    const V4c<R> Jc = load8(sh.J[sp[2]], (sp[3] & 4) ? R(-1) : R(1));
                    const cx<R> dac = dot2(Ja, Jc), dab = dot2(Ja, Jb), dbc = dot2(Jb, Jc);
                    const cx<R> hab = {dab.re * R(-0.5), dab.im * R(-0.5)};
                    const cx<R> hbc = {dbc.re * R(-0.5), dbc.im * R(-0.5)};
#pragma unroll
                    for (int mu = 0; mu < 4; ++mu) {
                        t.c[mu] = cfma(dac, Jb.c[mu], t.c[mu]);
                        t.c[mu] = cfma(hab, Jc.c[mu], t.c[mu]);
                        t.c[mu] = cfma(hbc, Ja.c[mu], t.c[mu]);
                    }
                }
                const R ig = sh.ig[T::cur_mask(c)];
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) t.c[mu] = cscale(t.c[mu], ig);
                store8(sh.J[c], t);
            }
            __syncthreads();
        }
#pragma unroll 1
        for (int ht = 0; ht < 2; ++ht) {
            for (int j = lane; j < 8; j += LPE) sh.Q[0][j] = sh.ub[ht][j];
            __syncthreads();
            // ---- quark line: prefixes by length, up to K - 2 (a prefix of length K - 1 fixes
            // its ordering, whose lane forms it below without storing it)
#pragma unroll 1
            for (int L = 1; L < K - 1; ++L) {
                for (int q = T::pre_levels(L) + lane; q < T::pre_levels(L + 1); q += LPE) {
                    V4c<R> psi{};
                    for (int s = 0; s < L; ++s) {
                        const short* sp = T::pre_split(q, s);
                        slash_row_add(load8(sh.Q[sp[0]], R(1)), load8(sh.J[sp[1]], sp[2] ? R(-1) : R(1)), psi);
                    }
                    const R* qp = sh.qp[T::pre_mask(q)];
                    const V4c<R> ql = V4c<R>{{{qp[0], R(0)}, {qp[1], R(0)}, {qp[2], qp[3]}, {qp[2], -qp[3]}}};
                    V4c<R> out;
#pragma unroll
                    for (int j = 0; j < 4; ++j) out.c[j] = cscale(psi.c[j], qp[4]);
                    slash_row_add(psi, ql, out);
                    store8(sh.Q[q], out);
                }
                __syncthreads();
            }
            // ---- amplitudes of the orderings
            for (int o = lane; o < T::NORD; o += LPE) {
                // the ordering's prefix of length K - 1 (all gluons but the last), in registers
                const short* last = T::ord_split(o, K - 1);
                const int q = last[0];
                V4c<R> psi{};
                for (int s = 0; s < K - 1; ++s) {
                    const short* sp = T::pre_split(q, s);
                    slash_row_add(load8(sh.Q[sp[0]], R(1)), load8(sh.J[sp[1]], sp[2] ? R(-1) : R(1)), psi);
                }
                const R* qp = sh.qp[T::pre_mask(q)];
                const V4c<R> ql = V4c<R>{{{qp[0], R(0)}, {qp[1], R(0)}, {qp[2], qp[3]}, {qp[2], -qp[3]}}};
                V4c<R> qlast;
#pragma unroll
                for (int j = 0; j < 4; ++j) qlast.c[j] = cscale(psi.c[j], qp[4]);
                slash_row_add(psi, ql, qlast);
                V4c<R> full{};
                for (int s = 0; s < K - 1; ++s) {
                    const short* sp = T::ord_split(o, s);
                    slash_row_add(load8(sh.Q[sp[0]], R(1)), load8(sh.J[sp[1]], sp[2] ? R(-1) : R(1)), full);
                }
                slash_row_add(qlast, load8(sh.J[last[1]], last[2] ? R(-1) : R(1)), full);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    cx<R> a = {R(0), R(0)};
#pragma unroll
                    for (int j = 0; j < 4; ++j) a = cfma(full.c[j], cx<R>{sh.vs[h][2 * j], sh.vs[h][2 * j + 1]}, a);
                    sh.A[h][o][0] = a.re;
                    sh.A[h][o][1] = a.im;
                }
            }
            __syncthreads();
            // ---- colour sum: lane takes the rows i = lane + r * LPE of C' (integer numerators;
            // C' symmetric, so row i is read as column i, coalesced across lanes) and runs over
            // the orderings j once for all its rows, each amplitude read from LDS once
            {
                constexpr int RP = (T::NORD + LPE - 1) / LPE;
                R y[RP][2][2];
#pragma unroll
                for (int r = 0; r < RP; ++r)
#pragma unroll
                    for (int h = 0; h < 2; ++h) y[r][h][0] = y[r][h][1] = R(0);
                for (int j = 0; j < T::NORD; ++j) {
                    R a[2][2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        a[h][0] = sh.A[h][j][0];
                        a[h][1] = sh.A[h][j][1];
                    }
#pragma unroll
                    for (int r = 0; r < RP; ++r) {
                        const R c = R(T::cnum(j, lane + r * LPE));      // 0 past the last row
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            y[r][h][0] = fma(c, a[h][0], y[r][h][0]);
                            y[r][h][1] = fma(c, a[h][1], y[r][h][1]);
                        }
                    }
                }
#pragma unroll
                for (int r = 0; r < RP; ++r) {
                    const int i = lane + r * LPE;
                    if (i < T::NORD) {
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            acc = fma(sh.A[h][i][0], y[r][h][0], fma(sh.A[h][i][1], y[r][h][1], acc));
                    }
                }
            }
            __syncthreads();
        }
    }
    double tot = double(acc);
#pragma unroll
    for (int m = LPE / 2; m > 0; m >>= 1) tot += __shfl_xor(tot, m);
    return tot;
}

// LPE lanes per event, 64 / LPE events per one-wave workgroup, each event its own LDS block
template <int K, typename R, int LPE>
__global__ __launch_bounds__(64) void k_me_bg(const double* __restrict__ p, int64_t n, R* __restrict__ out,
                                              double mt, double coupling)
{
    constexpr int EPB = 64 / LPE;
    __shared__ BgShared<K, R> sh[EPB];
    const int grp = threadIdx.x / LPE, lane = threadIdx.x % LPE;
    const int64_t e0 = (int64_t)blockIdx.x * EPB + grp;
    const int64_t e = e0 < n ? e0 : n - 1;      // a group past the end repeats the last event
    // the momenta go to LDS: the recursion indexes legs by table entries, which would put
    // a register copy in scratch memory
    for (int i = lane; i < (K + 2) * 4; i += LPE) sh[grp].pe[i / 4][i % 4] = p[i * n + e];
    __syncthreads();
    const double me = bg_event<K, R, LPE>(sh[grp].pe, mt, sh[grp], lane);
    if (lane == 0 && e0 < n) out[e0] = (R)(me * coupling * bg_norm_noalpha<K>());
}

}  // namespace mf
