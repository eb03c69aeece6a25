// Adjoint of the per-hit thin-film solve (reverse sweep with segment
// recomputation).  See gwg_device.h for the formulation.  Always double
// precision: the covector and the recomputed vectors carry the full
// conditioning of the stack.
#pragma once
#include "gwg_device.h"

namespace gwg {

struct V2d { double br, bi, cr, ci; };

__device__ inline void step_real_d(V2d& v, double C, double X, double Y)
{
    double br = fma(C, v.br, X * v.ci);
    double bi = fma(C, v.bi, -(X * v.cr));
    double cr = fma(C, v.cr, Y * v.bi);
    double ci = fma(C, v.ci, -(Y * v.br));
    v.br = br; v.bi = bi; v.cr = cr; v.ci = ci;
}

__device__ inline void step_cplx_d(V2d& v, cd C, cd X, cd Y)
{
    cd B = mk(v.br, v.bi), Cv = mk(v.cr, v.ci);
    cd mX = mk(X.im, -X.re), mY = mk(Y.im, -Y.re);
    cd b = cadd(cmul(C, B), cmul(mX, Cv));
    cd c = cadd(cmul(mY, B), cmul(C, Cv));
    v.br = b.re; v.bi = b.im; v.cr = c.re; v.ci = c.im;
}

// Entries of one layer for both polarizations.  Lossless: C real, X/Y real
// (imaginary parts zero).  Absorbing: complex.
struct LayerEnt { cd C, Xs, Ys, Xp, Yp; bool real; };

__device__ inline LayerEnt layer_entries(const LaneSlots3& sl, int s, bool cplx, double k0, double t)
{
    LayerEnt e;
    e.real = !cplx;
    if (!cplx) {
        double kq, xs, ys, xp, yp, C, S;
        sl.lossless(s, kq, xs, ys, xp, yp);
        layer_cs(kq, t, &C, &S);
        e.C = mk(C, 0.0);
        e.Xs = mk(S * xs, 0.0); e.Ys = mk(S * ys, 0.0);
        e.Xp = mk(S * xp, 0.0); e.Yp = mk(S * yp, 0.0);
    } else {
        double Pl[4];
        sl.absorbing(s, Pl);
        CTv<double> C, Xs, Ys, Xp, Yp;
        layer_cplx(Pl, k0, t, &C, &Xs, &Ys, &Xp, &Yp);
        e.C = mk(C.re, C.im); e.Xs = mk(Xs.re, Xs.im); e.Ys = mk(Ys.re, Ys.im);
        e.Xp = mk(Xp.re, Xp.im); e.Yp = mk(Yp.re, Yp.im);
    }
    return e;
}

__device__ inline void apply_layer(V2d& vs, V2d& vp, const LayerEnt& e)
{
    if (e.real) {
        step_real_d(vs, e.C.re, e.Xs.re, e.Ys.re);
        step_real_d(vp, e.C.re, e.Xp.re, e.Yp.re);
    } else {
        step_cplx_d(vs, e.C, e.Xs, e.Ys);
        step_cplx_d(vp, e.C, e.Xp, e.Yp);
    }
}

// u^T <- u^T M for M = [[C, -iX], [-iY, C]]:  u1' = u1 C - i u2 Y,  u2' = -i u1 X + u2 C
__device__ inline void cov_step(cd& u1, cd& u2, cd C, cd X, cd Y)
{
    cd mY = mk(Y.im, -Y.re), mX = mk(X.im, -X.re);
    cd n1 = cadd(cmul(u1, C), cmul(u2, mY));
    cd n2 = cadd(cmul(u1, mX), cmul(u2, C));
    u1 = n1; u2 = n2;
}

// u^T <- u^T M for a lossless layer, M = [[C, -iX], [-iY, C]] with real C, X, Y.
__device__ inline void cov_step_real(cd& u1, cd& u2, double C, double X, double Y)
{
    const double a = fma(u1.re, C, Y * u2.im), b = fma(u1.im, C, -(Y * u2.re));
    const double c = fma(u2.re, C, X * u1.im), d = fma(u2.im, C, -(X * u1.re));
    u1 = mk(a, b);
    u2 = mk(c, d);
}

// Adjoint of one mirror hit.  Adds d(2 Re(Gs c_s + Gp c_p))/dt_j for every
// layer into grad_row (this mirror's row of the calling wave's LDS
// accumulator, stack order), where c = r (reflect) or t (transmit).
// sl: this lane's slot table (N^2 of slot s: sl.nsq[2 s], sl.nsq[2 s + 1]).
// chk: this lane's checkpoint storage, component k of checkpoint c at
// chk[(c * 8 + k) * cstride].
__device__ inline void tmm_adjoint(const double* __restrict__ thk, const uint8_t* __restrict__ slot,
                                   int L, bool front, const LaneSlots3& sl, uint32_t cplx_mask, double k0,
                                   double kappa2, double eta0s, double eta0p, bool reflect, cd Gs, cd Gp,
                                   double* grad_row, double* __restrict__ chk, int64_t cstride)
{
    const double* nsq_c = sl.nsq;
    // 1) exit -> incident sweep, checkpoints w_{kSeg}, w_{2 kSeg}, ...
    V2d vs = { 1.0, 0.0, eta0s, 0.0 };
    V2d vp = { 1.0, 0.0, eta0p, 0.0 };
    for (int jj = L - 1; jj >= 0; --jj) {
        int idx = front ? jj : (L - 1 - jj);
        double t = thk[idx];
        if (t != 0.0) {
            int s = slot[idx];
            LayerEnt e = layer_entries(sl, s, (cplx_mask >> s) & 1u, k0, t);
            apply_layer(vs, vp, e);
        }
        if (jj > 0 && (jj % kSeg) == 0) {
            double* c = chk + (int64_t)(jj / kSeg) * 8 * cstride;
            c[0] = vs.br; c[cstride] = vs.bi; c[2 * cstride] = vs.cr; c[3 * cstride] = vs.ci;
            c[4 * cstride] = vp.br; c[5 * cstride] = vp.bi; c[6 * cstride] = vp.cr; c[7 * cstride] = vp.ci;
        }
    }
    // 2) cotangent row of the taken coefficient w.r.t. [B; C]
    cd u1s, u2s, u1p, u2p;
    {
        cd B = mk(vs.br, vs.bi), C = mk(vs.cr, vs.ci);
        cd den = cadd(cscale(B, eta0s), C);
        cd inv2 = cdiv(mk(1.0, 0.0), cmul(den, den));
        cd dB, dC;
        if (reflect) { dB = cscale(cmul(C, inv2), 2.0 * eta0s); dC = cscale(cmul(B, inv2), -2.0 * eta0s); }
        else { dB = cscale(inv2, -2.0 * eta0s * eta0s); dC = cscale(inv2, -2.0 * eta0s); }
        u1s = cmul(Gs, dB); u2s = cmul(Gs, dC);
    }
    {
        cd B = mk(vp.br, vp.bi), C = mk(vp.cr, vp.ci);
        cd den = cadd(cscale(B, eta0p), C);
        cd inv2 = cdiv(mk(1.0, 0.0), cmul(den, den));
        cd dB, dC;
        if (reflect) {   // r_p = -r_Mac
            dB = cscale(cmul(C, inv2), -2.0 * eta0p); dC = cscale(cmul(B, inv2), 2.0 * eta0p);
        } else { dB = cscale(inv2, -2.0 * eta0p * eta0p); dC = cscale(inv2, -2.0 * eta0p); }
        u1p = cmul(Gp, dB); u2p = cmul(Gp, dC);
    }
    // 3) incident -> exit covector sweep, segment by segment
    const int nseg = (L + kSeg - 1) / kSeg;
    for (int k = 0; k < nseg; ++k) {
        const int lo = k * kSeg;
        const int hi = min(lo + kSeg, L);
        V2d ws, wp;
        if (hi == L) {
            ws = V2d{ 1.0, 0.0, eta0s, 0.0 };
            wp = V2d{ 1.0, 0.0, eta0p, 0.0 };
        } else {
            const double* c = chk + (int64_t)(hi / kSeg) * 8 * cstride;
            ws = V2d{ c[0], c[cstride], c[2 * cstride], c[3 * cstride] };
            wp = V2d{ c[4 * cstride], c[5 * cstride], c[6 * cstride], c[7 * cstride] };
        }
        V2d segs[kSeg], segp[kSeg];
        double segC[kSeg], segS[kSeg];
#pragma unroll
        for (int i = kSeg - 1; i >= 0; --i) {
            const int jj = lo + i;
            segC[i] = 1.0; segS[i] = 0.0;
            if (jj < hi) {
                int idx = front ? jj : (L - 1 - jj);
                double t = thk[idx];
                int s = slot[idx];
                if (t != 0.0) {
                    if (!((cplx_mask >> s) & 1u)) {
                        double kq, xs, ys, xp, yp, C, S;
                        sl.lossless(s, kq, xs, ys, xp, yp);
                        layer_cs(kq, t, &C, &S);
                        segC[i] = C; segS[i] = S;
                        step_real_d(ws, C, S * xs, S * ys);
                        step_real_d(wp, C, S * xp, S * yp);
                    } else {
                        LayerEnt e = layer_entries(sl, s, true, k0, t);
                        apply_layer(ws, wp, e);
                    }
                }
                segs[i] = ws; segp[i] = wp;
            }
        }
#pragma unroll
        for (int i = 0; i < kSeg; ++i) {
            const int jj = lo + i;
            if (jj < hi) {
                int idx = front ? jj : (L - 1 - jj);
                double t = thk[idx];
                int s = slot[idx];
                bool cplx = (cplx_mask >> s) & 1u;
                // contraction u^T D w (D = -i k0 [[0, a], [b, 0]])
                cd Bs = mk(segs[i].br, segs[i].bi), Cs = mk(segs[i].cr, segs[i].ci);
                cd Bp = mk(segp[i].br, segp[i].bi), Cp = mk(segp[i].cr, segp[i].ci);
                cd As, Ap;
                if (!cplx) {
                    double n2 = nsq_c[2 * s];
                    double z = n2 - kappa2;
                    As = cadd(cmul(u1s, Cs), cscale(cmul(u2s, Bs), z));
                    Ap = cadd(cscale(cmul(u1p, Cp), z / n2), cscale(cmul(u2p, Bp), n2));
                } else {
                    cd N2 = mk(nsq_c[2 * s], nsq_c[2 * s + 1]);
                    cd z = csub(N2, mk(kappa2, 0.0));
                    As = cadd(cmul(u1s, Cs), cmul(z, cmul(u2s, Bs)));
                    Ap = cadd(cmul(cdiv(z, N2), cmul(u1p, Cp)), cmul(N2, cmul(u2p, Bp)));
                }
                // Re(-i k0 A) = k0 Im(A); dw/dt = 2 Re(...)
                double g = 2.0 * k0 * (As.im + Ap.im);
                atomicAdd(&grad_row[idx], g);
                // covector through layer jj
                if (t != 0.0) {
                    if (!cplx) {
                        double kq, xs, ys, xp, yp;
                        sl.lossless(s, kq, xs, ys, xp, yp);
                        const double C = segC[i], S = segS[i];
                        cov_step_real(u1s, u2s, C, S * xs, S * ys);
                        cov_step_real(u1p, u2p, C, S * xp, S * yp);
                    } else {
                        LayerEnt e = layer_entries(sl, s, true, k0, t);
                        cov_step(u1s, u2s, e.C, e.Xs, e.Ys);
                        cov_step(u1p, u2p, e.C, e.Xp, e.Yp);
                    }
                }
            }
        }
    }
}

// Cotangent row of the taken coefficient with respect to [B; C] at the
// incident side (Eq. 3 convention; r_p = -r_p of the characteristic matrix).
__device__ inline void coef_cotangent(const V2d& v, double eta0, bool reflect, bool p_pol, cd G, cd* u1, cd* u2)
{
    cd B = mk(v.br, v.bi), C = mk(v.cr, v.ci);
    cd den = cadd(cscale(B, eta0), C);
    cd inv2 = cdiv(mk(1.0, 0.0), cmul(den, den));
    cd dB, dC;
    if (reflect) {
        const double sg = p_pol ? -2.0 * eta0 : 2.0 * eta0;
        dB = cscale(cmul(C, inv2), sg);
        dC = cscale(cmul(B, inv2), -sg);
    } else {
        dB = cscale(inv2, -2.0 * eta0 * eta0);
        dC = cscale(inv2, -2.0 * eta0);
    }
    *u1 = cmul(G, dB);
    *u2 = cmul(G, dC);
}

// Adjoint of one mirror hit whose stack has no absorbing layer (every layer
// matrix has real C, X, Y).  Same contract as tmm_adjoint.  HC = false: no
// lane of the calling wave has an evanescent slot.  The contraction
// uses the slot parameters (x_s, y_s, x_p, y_p) = (1/q, q, q/N^2, N^2/q) for a
// propagating layer or (1/Q, -Q, -Q/N^2, N^2/Q) for an evanescent one
// (q = iQ), with sg = +1 or -1 respectively:
//     z = sg y_s^2,  z / N^2 = sg y_s x_p,  N^2 = sg y_s y_p.
template <bool HC = true>
__device__ inline void tmm_adjoint_lossless(const double* __restrict__ thk, const uint8_t* __restrict__ slot,
                                            int L, bool front, const LaneSlots3& sl, double k0,
                                            double eta0s, double eta0p, bool reflect, cd Gs, cd Gp,
                                            double* grad_row, double* __restrict__ chk, int64_t cstride,
                                            bool stored = false, int kseg = kSegL)
{
    // 1) exit -> incident sweep v_j = M_j v_{j+1}, checkpoints v_K, v_2K, ...
    //    (K = kseg, the hit's interval, the same as the forward solve's
    //    for a stored sweep): first the L % K layers above the last multiple of K,
    //    then whole groups of K layers, each ending in a checkpoint (group 0
    //    in none: v_0 stays in registers).  stored: the forward solve ran
    //    this sweep and left v_0 in block 0 and the checkpoints in blocks
    //    1.. (64-byte blocks, block g at chk + g cstride), with the same
    //    arithmetic: the half-period sine/cosine, whose sign (-1)^(sum n)
    //    is put back on each checkpoint and on v_0.
    if (L <= 0) return;
    const int K = kseg;
    V2d vs = { 1.0, 0.0, eta0s, 0.0 };
    V2d vp = { 1.0, 0.0, eta0p, 0.0 };
    double nsum = 0.0;
    auto sign_bit = [&]() { return (uint32_t)((int)nsum & 1) << 31; };
    auto layer_fwd = [&](int jj) {
        const int idx = front ? jj : (L - 1 - jj);
        double kq, xs, ys, xp, yp, C, S;
        sl.lossless(slot[idx], kq, xs, ys, xp, yp);
        layer_cs_half<double, HC>(kq, thk[idx], &C, &S, &nsum);   // t = 0 gives the identity exactly
        step_real_d(vs, C, S * xs, S * ys);
        step_real_d(vp, C, S * xp, S * yp);
    };
    auto checkpoint = [&](int g) {
        const uint32_t sb = sign_bit();
        double* c = chk + (int64_t)g * 8 * cstride;
        c[0] = flip_sign(vs.br, sb); c[cstride] = flip_sign(vs.bi, sb);
        c[2 * cstride] = flip_sign(vs.cr, sb); c[3 * cstride] = flip_sign(vs.ci, sb);
        c[4 * cstride] = flip_sign(vp.br, sb); c[5 * cstride] = flip_sign(vp.bi, sb);
        c[6 * cstride] = flip_sign(vp.cr, sb); c[7 * cstride] = flip_sign(vp.ci, sb);
    };
    // a stored block is 64 contiguous bytes, read whole
    auto read_block = [&](const double* c, V2d& a, V2d& b) {
        const double2* p = (const double2*)c;
        const double2 x0 = p[0], x1 = p[1], x2 = p[2], x3 = p[3];
        a = V2d{ x0.x, x0.y, x1.x, x1.y };
        b = V2d{ x2.x, x2.y, x3.x, x3.y };
    };
    if (stored) {
        read_block(chk, vs, vp);
    } else {
        const int ng = L / K;
        for (int jj = L - 1; jj >= ng * K; --jj) layer_fwd(jj);
        if (ng > 0 && ng * K < L) checkpoint(ng);    // v_{ng K}, after the top layers
        for (int g = ng - 1; g >= 0; --g) {
#pragma unroll 2
            for (int i = K - 1; i >= 0; --i) layer_fwd(g * K + i);
            if (g > 0) checkpoint(g);
        }
        const uint32_t sb = sign_bit();
        vs = V2d{ flip_sign(vs.br, sb), flip_sign(vs.bi, sb), flip_sign(vs.cr, sb), flip_sign(vs.ci, sb) };
        vp = V2d{ flip_sign(vp.br, sb), flip_sign(vp.bi, sb), flip_sign(vp.cr, sb), flip_sign(vp.ci, sb) };
    }
    // 2) cotangent rows of the taken coefficients
    cd u1s, u2s, u1p, u2p;
    coef_cotangent(vs, eta0s, reflect, false, Gs, &u1s, &u2s);
    coef_cotangent(vp, eta0p, reflect, true, Gp, &u1p, &u2p);
    // 3) incident -> exit covector sweep.  The state a layer's contraction
    //    needs, v_j, is walked down from the top of its segment (v_0 from the
    //    sweep, v_{kK} from checkpoint k) with the inverse layer matrix: a
    //    lossless layer, circular or hyperbolic, is unimodular with
    //    M^-1 = [[C, iX], [iY, C]], so one sine/cosine per layer serves the
    //    contraction, the covector step and the inverse step, and no
    //    per-segment state is kept.  Checkpoint k + 1 is loaded while segment
    //    k runs; each layer's LDS operands are loaded one layer ahead.
    //    The sines and cosines are the half-period ones, (-1)^n times the
    //    layer's own: after layers 0..j-1 the covector and the walked vector
    //    both carry the factor (-1)^(n_0 + ... + n_{j-1}), so their
    //    contraction is exact; a checkpoint (exact sign) joins the walk with
    //    that factor put on it.
    const double k2 = 2.0 * k0;
    double nsum_c = 0.0;                                // sum of the covector sweep's n so far
    V2d ws = vs, wp = vp, nws = vs, nwp = vp;
    auto load_chk = [&](int k) {
        const double* c = chk + (int64_t)k * (stored ? cstride : 8 * cstride);
        if (stored) {
            read_block(c, nws, nwp);
        } else {
            nws = V2d{ c[0], c[cstride], c[2 * cstride], c[3 * cstride] };
            nwp = V2d{ c[4 * cstride], c[5 * cstride], c[6 * cstride], c[7 * cstride] };
        }
    };
    if (K < L) load_chk(1);
    int gnext = 2;                                      // block of the checkpoint after the loaded one
    // Software pipeline over the layers, as in the forward sweep: layer
    // j+1's argument is reduced from slot parameters read one iteration
    // earlier, layer j+2's parameters and thickness are read, and layer
    // j+3's slot index.  Indices past the last layer stay at the last.
    using LT = LayerTrig<double, HC>;
    int idx = front ? 0 : L - 1;
    const int step = front ? 1 : -1;
    const int last = front ? L - 1 : 0;
    auto nxt = [&](int i) { return i == last ? i : i + step; };
    double kq, xs, ys, xp, yp;
    sl.lossless(slot[idx], kq, xs, ys, xp, yp);
    TrigArg ta = LT::reduce(kq, thk[idx]);              // t = 0 gives the identity exactly
    int idn = nxt(idx);
    double kq1, xs1, ys1, xp1, yp1;
    sl.lossless(slot[idn], kq1, xs1, ys1, xp1, yp1);
    double t1 = thk[idn];
    int idn2 = nxt(idn);
    int s2 = slot[idn2];
    for (int lo = 0; lo < L; lo += K) {
        if (lo > 0) {
            const uint32_t sb = (uint32_t)((int)nsum_c & 1) << 31;
            ws = V2d{ flip_sign(nws.br, sb), flip_sign(nws.bi, sb), flip_sign(nws.cr, sb), flip_sign(nws.ci, sb) };
            wp = V2d{ flip_sign(nwp.br, sb), flip_sign(nwp.bi, sb), flip_sign(nwp.cr, sb), flip_sign(nwp.ci, sb) };
            if (lo + K < L) load_chk(gnext);
            ++gnext;
        }
        const int hi = lo + K < L ? lo + K : L;
#pragma unroll 4
        for (int j = lo; j < hi; ++j) {
            const int idn3 = nxt(idn2);
            double kq2, xs2, ys2, xp2, yp2;
            sl.lossless(s2, kq2, xs2, ys2, xp2, yp2);
            const double t2 = thk[idn2];
            s2 = slot[idn3];
            const TrigArg ta1 = LT::reduce(kq1, t1);        // the next layer's (the last layer's again at the end)
            double C, S;
            LT::eval(ta, &C, &S, &nsum_c);
            const double sXs = S * xs, sYs = S * ys, sXp = S * xp, sYp = S * yp;
            const double gys = (HC && kq < 0.0) ? -ys : ys;       // sg y_s (an evanescent layer: sg = -1)
            // Im(u^T D w) summed over s and p, D = -i k0 [[0, a], [b, 0]]
            // (fused multiply-adds written out: the library builds without
            // contraction)
            const double i_s1 = fma(u1s.re, ws.ci, u1s.im * ws.cr);   // Im(u1s C_s)
            const double i_s2 = fma(u2s.re, ws.bi, u2s.im * ws.br);   // Im(u2s B_s)
            const double i_p1 = fma(u1p.re, wp.ci, u1p.im * wp.cr);   // Im(u1p C_p)
            const double i_p2 = fma(u2p.re, wp.bi, u2p.im * wp.br);   // Im(u2p B_p)
            const double g = k2 * fma(gys, fma(yp, i_p2, fma(xp, i_p1, ys * i_s2)), i_s1);
            atomicAdd(&grad_row[idx], g);
            cov_step_real(u1s, u2s, C, sXs, sYs);
            cov_step_real(u1p, u2p, C, sXp, sYp);
            step_real_d(ws, C, -sXs, -sYs);
            step_real_d(wp, C, -sXp, -sYp);
            idx = idn; ta = ta1; kq = kq1; xs = xs1; ys = ys1; xp = xp1; yp = yp1;
            idn = idn2; kq1 = kq2; xs1 = xs2; ys1 = ys2; xp1 = xp2; yp1 = yp2; t1 = t2;
            idn2 = idn3;
        }
    }
}

}  // namespace gwg
