// Reverse-mode derivatives (vector-Jacobian products) of the step's
// pointwise functions, written by hand from the forward formulas in
// ppm_math.h.  Every function recomputes its forward values, takes every
// branch (limiter case, floor, wave side, shock/fan) as the forward did —
// the derivative of the step with its branch decisions frozen — and
// accumulates the input adjoints (+=) from the output adjoints.
#pragma once

#include "ppm_math.h"

namespace ppm {

// The value x, hidden from the compiler's common-subexpression elimination
// (an empty asm statement that claims to modify x, no instruction).  A
// reverse pass that recomputes a forward quantity from opaque(x) gets a
// fresh value; without it the compiler would reuse the forward pass's value
// and keep it live in registers from the forward to the reverse pass.
template <class S> PPM_HD S opaque(S x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x));
#endif
  return x;
}

// --------------------------------------------------------------- flux ------
// F = flux of the rotated state g = (rho, u_n, p, u_t1, u_t2) along d (xyz
// component order).  gb += (dF/dg)^T Fb.
template <int d, class S>
PPM_HD void flux_vjp(const S g[5], const Gas<S>& G, const S Fb[5], S gb[5]) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const S r = g[0], u = g[1], p = g[2], v1 = g[3], v2 = g[4];
  const S m = r * u;
  const S K = (u * u + v1 * v1) + v2 * v2;
  const S e = p * G.gm1inv + HALF * r * K;
  const S f0 = Fb[0], fn = Fb[1 + d], f1 = Fb[1 + t1], f2 = Fb[1 + t2], fe = Fb[4];
  const S mb = f0 + fn * u + f1 * v1 + f2 * v2;
  S ub = fn * m + fe * (e + p);
  S pb = fn + fe * u;
  const S eb = fe * u;
  S v1b = f1 * m, v2b = f2 * m;
  pb += eb * G.gm1inv;
  S rb = eb * HALF * K;
  ub += eb * r * u;
  v1b += eb * r * v1;
  v2b += eb * r * v2;
  rb += mb * u;
  ub += mb * r;
  gb[0] += rb; gb[1] += ub; gb[2] += pb; gb[3] += v1b; gb[4] += v2b;
}

// -------------------------------------------------------- fan sampling -----
// Reverse of sample_side (left orientation).  Adjoints of the outputs
// (r_, u_, p_) in (rb_, ub_, pb_); accumulates into the adjoints of
// ro, uo, po, C, iW, us and p (the shock speed uses W only in a test).
template <class S>
PPM_HD void sample_side_vjp(S ro, S uo, S po, S C, S W, S iW, S us, S p, const Gas<S>& G, S rb_, S ub_,
                            S pb_, S& rob, S& uob, S& pob, S& Cb, S& iWb, S& usb, S& pb) {
  const S irho = qdiv(ONE, ro);
  const S vstar = irho - (p - po) * (iW * iW);
  S rs = qdiv(ONE, vstar), ivs = vstar;
  bool fl = false;
  if (!(vstar > S(0)) || rs < G.small_dens) { fl = true; rs = G.small_dens; ivs = G.ismall_dens; }
  const S cst = sqrt_phys(G.gamma * p * ivs);
  const S co = C * irho;
  S rsb = S(0), cstb = S(0), cob = S(0), irhob = S(0), ivsb = S(0);
  if (p > po) {
    const S sh = uo - W * irho;
    if (!(sh >= S(0))) { rsb += rb_; usb += ub_; pb += pb_; }
    else { rob += rb_; uob += ub_; pob += pb_; }
  } else {
    const S hd = uo - co, tl = us - cst;
    if (hd >= S(0)) {
      rob += rb_; uob += ub_; pob += pb_;
    } else if (tl <= S(0)) {
      rsb += rb_; usb += ub_; pb += pb_;
    } else {
      const S D = tl - hd;
      const S iD = qdiv(ONE, D);
      const S w = -hd * iD;
      const S wb = rb_ * (rs - ro) + ub_ * (us - uo) + pb_ * (p - po);
      rob += (ONE - w) * rb_;
      rsb += w * rb_;
      uob += (ONE - w) * ub_;
      usb += w * ub_;
      pob += (ONE - w) * pb_;
      pb += w * pb_;
      const S hdb = -wb * tl * iD * iD;
      const S tlb = wb * hd * iD * iD;
      uob += hdb;
      cob -= hdb;
      usb += tlb;
      cstb -= tlb;
    }
  }
  // cst = sqrt(gamma p ivs), co = C / rho
  if (cstb != S(0)) {
    const S h = cstb * HALF / cst;
    pb += h * G.gamma * ivs;
    ivsb += h * G.gamma * p;
  }
  Cb += cob * irho;
  irhob += cob * C;
  // rs = 1 / vstar and ivs = vstar (floor frozen)
  const S vstarb = fl ? S(0) : -rsb * rs * rs + ivsb;
  irhob += vstarb;
  pb -= vstarb * (iW * iW);
  pob += vstarb * (iW * iW);
  iWb -= vstarb * (p - po) * TWO * iW;
  rob -= irhob * irho * irho;
}

// Newton steps whose input pressures the Riemann reverse keeps in registers
// (the reverse of such a step recomputes its forward from that pressure).
constexpr int RIEM_KEEP = 3;

// One Newton step of the two-shock iteration, forward (returns the new p).
template <class S>
PPM_HD S riem_iter(S p, S cl, S cr, S pl, S pr, S ul, S ur, S ipl, S ipr, const Gas<S>& G) {
  const S wl = cl * sqrt_wave(ONE + G.beta * (p * ipl - ONE));
  const S wr = cr * sqrt_wave(ONE + G.beta * (p * ipr - ONE));
  S iwl, iwr;
  pair_recip(wl, wr, iwl, iwr);
  const S xl = cl * iwl, xr = cr * iwr;
  const S izl = HALF * iwl * (ONE + xl * xl);
  const S izr = HALF * iwr * (ONE + xr * xr);
  const S usl = ul - (p - pl) * iwl;
  const S usr = ur + (p - pr) * iwr;
  const S pn = p - qdiv(usr - usl, izl + izr);
  return smax(pn, G.small_pres);
}

// What the reverse of one Newton step needs from its forward evaluation.
template <class S> struct RiemIt {
  S p, sl, sr, iwl, iwr;  // input p, sqrt(a_s), 1/W_s
  bool floored;           // the output was bound by the pressure floor
};

// One Newton step, forward (the same arithmetic as riem_iter), recording
// what its reverse needs.
template <class S>
PPM_HD S riem_iter_rec(S p, S cl, S cr, S pl, S pr, S ul, S ur, S ipl, S ipr, const Gas<S>& G, RiemIt<S>& r) {
  const S sl = sqrt_wave(ONE + G.beta * (p * ipl - ONE));
  const S sr = sqrt_wave(ONE + G.beta * (p * ipr - ONE));
  const S wl = cl * sl, wr = cr * sr;
  S iwl, iwr;
  pair_recip(wl, wr, iwl, iwr);
  const S xl = cl * iwl, xr = cr * iwr;
  const S izl = HALF * iwl * (ONE + xl * xl);
  const S izr = HALF * iwr * (ONE + xr * xr);
  const S usl = ul - (p - pl) * iwl;
  const S usr = ur + (p - pr) * iwr;
  const S pn = p - qdiv(usr - usl, izl + izr);
  r.p = p;
  r.sl = sl;
  r.sr = sr;
  r.iwl = iwl;
  r.iwr = iwr;
  r.floored = pn < G.small_pres;
  return smax(pn, G.small_pres);
}

// Reverse of one Newton step from its record: pnb = adjoint of the output
// p; returns the adjoint of the input p and accumulates the others.
template <class S>
PPM_HD S riem_iter_vjp_rec(const RiemIt<S>& r, S cl, S cr, S pl, S pr, S ul, S ur, S ipl, S ipr, const Gas<S>& G,
                           S pnb, S& clb, S& crb, S& plb, S& prb, S& ulb, S& urb, S& iplb, S& iprb) {
  if (r.floored) return S(0);  // floor bound: the output does not depend on p
  const S p = r.p, sl = r.sl, sr = r.sr, iwl = r.iwl, iwr = r.iwr;
  const S xl = cl * iwl, xr = cr * iwr;
  const S izl = HALF * iwl * (ONE + xl * xl);
  const S izr = HALF * iwr * (ONE + xr * xr);
  const S usl = ul - (p - pl) * iwl;
  const S usr = ur + (p - pr) * iwr;
  const S dU = usr - usl, Q = izl + izr;
  S pb = pnb;
  const S iQ = qdiv(ONE, Q);
  const S dUb = -pnb * iQ;
  const S Qb = pnb * dU * iQ * iQ;
  const S usrb = dUb, uslb = -dUb;
  ulb += uslb;
  pb -= uslb * iwl;
  plb += uslb * iwl;
  S iwlb = -uslb * (p - pl);
  urb += usrb;
  pb += usrb * iwr;
  prb -= usrb * iwr;
  S iwrb = usrb * (p - pr);
  iwlb += Qb * HALF * (ONE + xl * xl);
  const S xlb = Qb * iwl * xl;
  iwrb += Qb * HALF * (ONE + xr * xr);
  const S xrb = Qb * iwr * xr;
  clb += xlb * iwl;
  iwlb += xlb * cl;
  crb += xrb * iwr;
  iwrb += xrb * cr;
  const S wlb = -iwlb * iwl * iwl, wrb = -iwrb * iwr * iwr;
  clb += wlb * sl;
  crb += wrb * sr;
  // cl / (2 sl) = cl^2 / (2 wl)
  const S alb = wlb * HALF * cl * cl * iwl, arb = wrb * HALF * cr * cr * iwr;
  pb += alb * G.beta * ipl + arb * G.beta * ipr;
  iplb += alb * G.beta * p;
  iprb += arb * G.beta * p;
  return pb;
}

// Reverse of one Newton step with its forward recomputed from the input p.
template <class S>
PPM_HD S riem_iter_vjp(S p, S cl, S cr, S pl, S pr, S ul, S ur, S ipl, S ipr, const Gas<S>& G, S pnb, S& clb,
                       S& crb, S& plb, S& prb, S& ulb, S& urb, S& iplb, S& iprb) {
  RiemIt<S> r;
  (void)riem_iter_rec(p, cl, cr, pl, pr, ul, ur, ipl, ipr, G, r);
  return riem_iter_vjp_rec(r, cl, cr, pl, pr, ul, ur, ipl, ipr, G, pnb, clb, crb, plb, prb, ulb, urb, iplb, iprb);
}

// Reverse of riemann<d>: Fb = adjoint of the flux; accumulates Lb, Rb.
// REC: keep each kept Newton step's full record in registers (no forward
// recomputation in the reverse sweep, more registers) instead of its input
// pressure alone.
template <int d, bool REC = false, class S>
PPM_HD void riemann_vjp(const S L[5], const S R[5], const Gas<S>& G, const S Fb[5], S Lb[5], S Rb[5]) {
  constexpr int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
  const S rl = L[0], ul = L[1 + d], pl = L[4];
  const S rr = R[0], ur = R[1 + d], pr = R[4];
  const S cl = sqrt_phys(G.gamma * pl * rl);
  const S cr = sqrt_phys(G.gamma * pr * rr);
  const S N0 = (cr * pl + cl * pr) + (cl * cr) * (ul - ur);
  const S D0 = cl + cr;
  const S p0r = qdiv(N0, D0);
  const bool fl0 = p0r < G.small_pres;
  const S p0 = smax(p0r, G.small_pres);
  const S ipl = qdiv(ONE, pl), ipr = qdiv(ONE, pr);
  // the input pressures of the first RIEM_KEEP Newton steps (with REC their
  // full records) are kept for the reverse sweep (fully unrolled, so they
  // stay in registers); later steps are recomputed from the output of the
  // last kept one
  S pin[RIEM_KEEP];
  RiemIt<S> rec[REC ? RIEM_KEEP : 1];
  S pst = p0;
#pragma unroll
  for (int it = 0; it < RIEM_KEEP; ++it)
    if (it < G.iters) {
      pin[it] = pst;
      if constexpr (REC) pst = riem_iter_rec(pst, cl, cr, pl, pr, ul, ur, ipl, ipr, G, rec[it]);
      else pst = riem_iter(pst, cl, cr, pl, pr, ul, ur, ipl, ipr, G);
    }
  const S pkeep = pst;
  for (int it = RIEM_KEEP; it < G.iters; ++it) pst = riem_iter(pst, cl, cr, pl, pr, ul, ur, ipl, ipr, G);
  const S all = ONE + G.beta * (pst * ipl - ONE), alr = ONE + G.beta * (pst * ipr - ONE);
  const S sl = sqrt_wave(all), sr = sqrt_wave(alr);
  const S wl = cl * sl, wr = cr * sr;
  S iwl, iwr;
  pair_recip(wl, wr, iwl, iwr);
  const S NU = (wl * ul + wr * ur) + (pl - pr), DU = wl + wr;
  const S us = qdiv(NU, DU);

  // forward sample -> Godunov state g, then the flux adjoint
  S g[5];
  int dummy = 0;
  if (us != S(0)) {
    const bool left = us > S(0);
    S r_, u_, p_;
    if (left) sample_side(rl, ul, pl, cl, wl, iwl, us, pst, G, r_, u_, p_, dummy);
    else sample_side(rr, -ur, pr, cr, wr, iwr, -us, pst, G, r_, u_, p_, dummy);
    g[0] = r_; g[1] = left ? u_ : -u_; g[2] = p_;
    g[3] = left ? L[1 + t1] : R[1 + t1];
    g[4] = left ? L[1 + t2] : R[1 + t2];
  } else {
    S ra, ua, pa, rb, ub, pb;
    sample_side(rl, ul, pl, cl, wl, iwl, us, pst, G, ra, ua, pa, dummy);
    sample_side(rr, -ur, pr, cr, wr, iwr, -us, pst, G, rb, ub, pb, dummy);
    ub = -ub;
    g[0] = HALF * (ra + rb); g[1] = HALF * (ua + ub); g[2] = HALF * (pa + pb);
    g[3] = HALF * (L[1 + t1] + R[1 + t1]);
    g[4] = HALF * (L[1 + t2] + R[1 + t2]);
  }
  S gb[5] = {S(0), S(0), S(0), S(0), S(0)};
  flux_vjp<d>(g, G, Fb, gb);

  S rlb = S(0), ulb = S(0), plb = S(0), clb = S(0), iwlb = S(0);
  S rrb = S(0), urb = S(0), prb = S(0), crb = S(0), iwrb = S(0);
  S usb = S(0), pstb = S(0);
  if (us != S(0)) {
    // one side sampled: its inputs selected, its adjoints added to that side
    const bool left = us > S(0);
    const S sg = left ? ONE : -ONE;
    S rob = S(0), uob = S(0), pob = S(0), Cb = S(0), iWb = S(0), usbs = S(0);
    sample_side_vjp(left ? rl : rr, left ? ul : -ur, left ? pl : pr, left ? cl : cr, left ? wl : wr,
                    left ? iwl : iwr, left ? us : -us, pst, G, gb[0], sg * gb[1], gb[2], rob, uob, pob, Cb, iWb,
                    usbs, pstb);
    usb = sg * usbs;
    // selects, not branches, so that the compiler keeps the adjoints in registers
    rlb = left ? rob : S(0); ulb = left ? uob : S(0); plb = left ? pob : S(0);
    clb = left ? Cb : S(0); iwlb = left ? iWb : S(0);
    rrb = left ? S(0) : rob; urb = left ? S(0) : -uob; prb = left ? S(0) : pob;
    crb = left ? S(0) : Cb; iwrb = left ? S(0) : iWb;
    Lb[1 + t1] += left ? gb[3] : S(0);
    Lb[1 + t2] += left ? gb[4] : S(0);
    Rb[1 + t1] += left ? S(0) : gb[3];
    Rb[1 + t2] += left ? S(0) : gb[4];
  } else {
    const S h0 = HALF * gb[0], h1 = HALF * gb[1], h2 = HALF * gb[2];
    sample_side_vjp(rl, ul, pl, cl, wl, iwl, us, pst, G, h0, h1, h2, rlb, ulb, plb, clb, iwlb, usb, pstb);
    S uob = S(0), usbm = S(0);
    sample_side_vjp(rr, -ur, pr, cr, wr, iwr, -us, pst, G, h0, -h1, h2, rrb, uob, prb, crb, iwrb, usbm, pstb);
    urb -= uob;
    usb -= usbm;
    Lb[1 + t1] += HALF * gb[3];
    Rb[1 + t1] += HALF * gb[3];
    Lb[1 + t2] += HALF * gb[4];
    Rb[1 + t2] += HALF * gb[4];
  }
  // us = NU / DU
  const S iDU = qdiv(ONE, DU);
  const S NUb = usb * iDU, DUb = -usb * us * iDU;
  S wlb = NUb * ul + DUb, wrb = NUb * ur + DUb;
  ulb += NUb * wl;
  urb += NUb * wr;
  plb += NUb;
  prb -= NUb;
  wlb -= iwlb * iwl * iwl;
  wrb -= iwrb * iwr * iwr;
  clb += wlb * sl;
  crb += wrb * sr;
  S iplb = S(0), iprb = S(0);
  {
    const S alb = wlb * HALF * cl * cl * iwl, arb = wrb * HALF * cr * cr * iwr;
    pstb += alb * G.beta * ipl + arb * G.beta * ipr;
    iplb += alb * G.beta * pst;
    iprb += arb * G.beta * pst;
  }
  // Newton iterations in reverse
  S pb = pstb;
  for (int k = G.iters - 1; k >= RIEM_KEEP; --k) {
    S pk = pkeep;
    for (int j = RIEM_KEEP; j < k; ++j) pk = riem_iter(pk, cl, cr, pl, pr, ul, ur, ipl, ipr, G);
    pb = riem_iter_vjp(pk, cl, cr, pl, pr, ul, ur, ipl, ipr, G, pb, clb, crb, plb, prb, ulb, urb, iplb, iprb);
  }
#pragma unroll
  for (int k = RIEM_KEEP - 1; k >= 0; --k)
    if (k < G.iters) {
      if constexpr (REC)
        pb = riem_iter_vjp_rec(rec[k], cl, cr, pl, pr, ul, ur, ipl, ipr, G, pb, clb, crb, plb, prb, ulb, urb, iplb,
                               iprb);
      else
        pb = riem_iter_vjp(opaque(pin[k]), cl, cr, pl, pr, ul, ur, ipl, ipr, G, pb, clb, crb, plb, prb, ulb, urb,
                           iplb, iprb);
    }
  // acoustic guess (floor frozen)
  if (!fl0) {
    const S iD0 = qdiv(ONE, D0);
    const S N0b = pb * iD0, D0b = -pb * p0r * iD0;
    crb += N0b * (pl + cl * (ul - ur));
    plb += N0b * cr;
    clb += N0b * (pr + cr * (ul - ur));
    prb += N0b * cl;
    ulb += N0b * (cl * cr);
    urb -= N0b * (cl * cr);
    clb += D0b;
    crb += D0b;
  }
  plb -= iplb * ipl * ipl;
  prb -= iprb * ipr * ipr;
  // cl^2 = gamma pl rl: d cl = gamma (rl d pl + pl d rl) / (2 cl)
  const S hl = clb * HALF * G.gamma / cl, hr = crb * HALF * G.gamma / cr;
  plb += hl * rl;
  rlb += hl * pl;
  prb += hr * rr;
  rrb += hr * pr;
  Lb[0] += rlb; Lb[1 + d] += ulb; Lb[4] += plb;
  Rb[0] += rrb; Rb[1 + d] += urb; Rb[4] += prb;
}

// ----------------------------------------------------------- conversions ---
// U = cons(q): qb += (dU/dq)^T Ub.
template <class S>
PPM_HD void prim_to_cons_vjp(const S q[5], const Gas<S>& G, const S Ub[5], S qb[5]) {
  const S K = (q[1] * q[1] + q[2] * q[2]) + q[3] * q[3];
  qb[0] += Ub[0] + Ub[1] * q[1] + Ub[2] * q[2] + Ub[3] * q[3] + Ub[4] * HALF * K;
  qb[1] += Ub[1] * q[0] + Ub[4] * q[0] * q[1];
  qb[2] += Ub[2] * q[0] + Ub[4] * q[0] * q[2];
  qb[3] += Ub[3] * q[0] + Ub[4] * q[0] * q[3];
  qb[4] += Ub[4] * G.gm1inv;
}

// Shared tail of the primitive-conversion adjoints: from (rb, ub, vb, wb, pb)
// of q = (r, U1/r, U2/r, U3/r, gm1 (U4 - r K / 2)) to Ub (pressure floor
// already applied by the caller, density floor handled by the caller).
template <class S>
PPM_HD void prim_tail_vjp(S r, S u, S v, S w, const Gas<S>& G, S rb, S ub, S vb, S wb, S pb, S Ub[5], bool rfloor) {
  const S K = (u * u + v * v) + w * w;
  Ub[4] += G.gm1 * pb;
  const S keb = -G.gm1 * pb;
  rb += keb * HALF * K;
  ub += keb * r * u;
  vb += keb * r * v;
  wb += keb * r * w;
  const S ir = qdiv(ONE, r);
  Ub[1] += ub * ir;
  Ub[2] += vb * ir;
  Ub[3] += wb * ir;
  rb -= (ub * u + vb * v + wb * w) * ir;
  if (!rfloor) Ub[0] += rb;
}

// q = cons_to_prim_floor(U): Ub += (dq/dU)^T qb.
template <class S>
PPM_HD void cons_to_prim_floor_vjp(const S U[5], const Gas<S>& G, const S qb[5], S Ub[5]) {
  const bool rfl = U[0] < G.small_dens;
  const S r = smax(U[0], G.small_dens);
  const S ir0 = qdiv(ONE, r);
  const S u = U[1] * ir0, v = U[2] * ir0, w = U[3] * ir0;
  const S ke = HALF * r * ((u * u + v * v) + w * w);
  const S p = G.gm1 * (U[4] - ke);
  const S pb = (p < G.small_pres) ? S(0) : qb[4];
  prim_tail_vjp(r, u, v, w, G, qb[0], qb[1], qb[2], qb[3], pb, Ub, rfl);
}

// cons_to_prim_floor (same arithmetic), also returning its two floor
// decisions for the reverse.
template <class S>
PPM_HD void cons_to_prim_dec(const S U[5], const Gas<S>& G, S q[5], bool& rfl, bool& pfl) {
  rfl = U[0] < G.small_dens;
  const S r = smax(U[0], G.small_dens);
  const S ir = qdiv(ONE, r);
  const S u = U[1] * ir, v = U[2] * ir, w = U[3] * ir;
  const S ke = HALF * r * ((u * u + v * v) + w * w);
  const S p = G.gm1 * (U[4] - ke);
  pfl = p < G.small_pres;
  q[0] = r; q[1] = u; q[2] = v; q[3] = w; q[4] = smax(p, G.small_pres);
}

// Reverse of cons_to_prim_floor from its outputs q and floor decisions.
template <class S>
PPM_HD void cons_to_prim_vjp_q(const S q[5], bool rfl, bool pfl, const Gas<S>& G, const S qb[5], S Ub[5]) {
  prim_tail_vjp(q[0], q[1], q[2], q[3], G, qb[0], qb[1], qb[2], qb[3], pfl ? S(0) : qb[4], Ub, rfl);
}

// Cell conversion of a stored zone (rho, u, v, w, p, c): Ub += J^T qb.
template <class S>
PPM_HD void prim_cell_vjp(const S U[5], const Gas<S>& G, const S qb[6], S Ub[5]) {
  const S r = U[0];
  const S u = U[1] / r, v = U[2] / r, w = U[3] / r;
  const S ke = HALF * r * ((u * u + v * v) + w * w);
  const S praw = G.gm1 * (U[4] - ke);
  const bool pfl = praw < G.small_pres;
  const S p = smax(praw, G.small_pres);
  const S c = ssqrt(G.gamma * p / r);
  const S h = qb[5] * HALF / (r * c);
  S pb = qb[4] + h * G.gamma;
  const S rb = qb[0] - h * c * c;
  if (pfl) pb = S(0);
  prim_tail_vjp(r, u, v, w, G, rb, qb[1], qb[2], qb[3], pb, Ub, false);
}

// --------------------------------------------------------------- PPM -------
template <class S>
PPM_HD void ppm_slope_vjp(S am, S a0, S ap, int limiter, S sb, S& amb, S& a0b, S& apb) {
  const S dc = HALF * (ap - am);
  S dcb = S(0);
  if (!limiter) {
    dcb = sb;
  } else {
    const S dl = a0 - am, dr = ap - a0;
    if (!same_sign(dl, dr)) return;
    const S A = sabs(dc), B = TWO * sabs(dl), C = TWO * sabs(dr);
    const S m1 = smin(A, B);
    const bool selA = !(B < A);
    const bool selm1 = !(C < m1);
    const S Mb = flipsign(sb, dc);
    S Ab = S(0), Bb = S(0), Cb = S(0);
    if (selm1) {
      if (selA) Ab = Mb; else Bb = Mb;
    } else {
      Cb = Mb;
    }
    // dc, dl, dr are nonzero here: the sign flips are the products with their signs
    dcb = flipsign(Ab, dc);
    const S dlb = TWO * flipsign(Bb, dl);
    const S drb = TWO * flipsign(Cb, dr);
    a0b += dlb - drb;
    amb -= dlb;
    apb += drb;
  }
  apb += HALF * dcb;
  amb -= HALF * dcb;
}

// Reverse of ppm_parabola: (aLb, aRb, a6b) -> ab[0..4] (stencil i-2..i+2), phib.
template <class S>
PPM_HD void ppm_parabola_vjp(const S a[5], S phi, const Gas<S>& G, S aLb, S aRb, S a6b, S ab[5], S& phib) {
  const S sm = ppm_slope(a[0], a[1], a[2], G.limiter);
  const S s0 = ppm_slope(a[1], a[2], a[3], G.limiter);
  const S sp = ppm_slope(a[2], a[3], a[4], G.limiter);
  const S a0 = a[2];
  const S aL = HALF * (a[1] + a0) - (s0 - sm) * SIXTH;
  const S aR = HALF * (a0 + a[3]) - (sp - s0) * SIXTH;
  S aL1 = aL, aR1 = aR;
  if (G.limiter && G.flattening) {
    const S omp = ONE - phi;
    aL1 = phi * aL + omp * a0;
    aR1 = phi * aR + omp * a0;
  }
  // a6 = 6 a0 - 3 (aL2 + aR2)
  S aL2b = aLb - THREE * a6b, aR2b = aRb - THREE * a6b;
  ab[2] += SIX * a6b;
  S aL1b = aL2b, aR1b = aR2b;
  if (G.limiter) {
    if (!same_sign(aR1 - a0, a0 - aL1)) {
      ab[2] += aL2b + aR2b;
      aL1b = S(0);
      aR1b = S(0);
    } else {
      bool hi, lo;
      cw_overshoot(aR1 - aL1, a0 - HALF * (aL1 + aR1), hi, lo);
      if (hi) {
        ab[2] += THREE * aL2b;
        aR1b = aR2b - TWO * aL2b;
        aL1b = S(0);
      } else if (lo) {
        ab[2] += THREE * aR2b;
        aL1b = aL2b - TWO * aR2b;
        aR1b = S(0);
      }
    }
  }
  S aLe = aL1b, aRe = aR1b;
  if (G.limiter && G.flattening) {
    const S omp = ONE - phi;
    aLe = phi * aL1b;
    aRe = phi * aR1b;
    ab[2] += omp * (aL1b + aR1b);
    phib += aL1b * (aL - a0) + aR1b * (aR - a0);
  }
  // edges
  ab[1] += HALF * aLe;
  ab[2] += HALF * aLe + HALF * aRe;
  ab[3] += HALF * aRe;
  const S smb = aLe * SIXTH;
  const S s0b = -aLe * SIXTH + aRe * SIXTH;
  const S spb = -aRe * SIXTH;
  ppm_slope_vjp(a[0], a[1], a[2], G.limiter, smb, ab[0], ab[1], ab[2]);
  ppm_slope_vjp(a[1], a[2], a[3], G.limiter, s0b, ab[1], ab[2], ab[3]);
  ppm_slope_vjp(a[2], a[3], a[4], G.limiter, spb, ab[2], ab[3], ab[4]);
}

// Reverse of ppm_ip / ppm_im for a given Courant number (adjoint Ib).
template <class S>
PPM_HD void ppm_ip_vjp(S da, S a6, S sg, S Ib, S& aRb, S& dab, S& a6b, S& sgb) {
  const S f = ONE - TWO3 * sg;
  const S B = da - f * a6;
  const S h = HALF * sg;
  aRb += Ib;
  const S hb = -Ib * B, Bb = -Ib * h;
  dab += Bb;
  const S fb = -Bb * a6;
  a6b -= Bb * f;
  sgb += HALF * hb - TWO3 * fb;
}
template <class S>
PPM_HD void ppm_im_vjp(S da, S a6, S sg, S Ib, S& aLb, S& dab, S& a6b, S& sgb) {
  const S f = ONE - TWO3 * sg;
  const S B = da + f * a6;
  const S h = HALF * sg;
  aLb += Ib;
  const S hb = Ib * B, Bb = Ib * h;
  dab += Bb;
  a6b += Bb * f;
  const S fb = Bb * a6;
  sgb += HALF * hb - TWO3 * fb;
}

// ------------------------------------------------------------ tracing ------
// The tracing couples density, normal velocity and pressure through the
// three waves; each transverse velocity only moves with the middle wave, so
// its edge values depend on its own parabola and the wave speeds alone.
// The reverse is split the same way (fewer values live at once).

// Reverse of trace_zone<d> for the coupled fields 0, 1 + d and 4:
// (qpb, qmb) of those fields -> their (aLb, aRb, a6b), rb, unb, cb.  lamb:
// the wave-speed adjoints the transverse fields' reverses left (added here).
template <int d, class S>
PPM_HD void trace_zone_vjp(const S aL[5], const S aR[5], const S a6[5], S r, S un, S c, S dtdx, const Gas<S>& G,
                           const S qpb[5], const S qmb[5], const S lambt[3], S aLb[5], S aRb[5], S a6b[5], S& rb,
                           S& unb, S& cb) {
  constexpr int mn = 1 + d;
  constexpr int fm[3] = {0, mn, 4};
  S da[5], dab[5];
#pragma unroll
  for (int i = 0; i < 3; ++i) { da[fm[i]] = aR[fm[i]] - aL[fm[i]]; dab[fm[i]] = S(0); }
  const S rc = r * c, c2 = c * c, ic2 = qdiv(ONE, c2), hic2 = HALF * ic2, cor = qdiv(c, r);
  const S lam[3] = {un - c, un, un + c};
  const S zero = S(0);
  S rcb = zero, c2b = zero, ic2b = zero, hic2b = zero, corb = zero;
  S lamb[3] = {lambt[0], lambt[1], lambt[2]};

  for (int side = 0; side < 2; ++side) {
    const bool hi = side == 0;
    S sg[3], sgb[3] = {zero, zero, zero};
    for (int k = 0; k < 3; ++k) sg[k] = smax(hi ? lam[k] : -lam[k], zero) * dtdx;
    const int kref = hi ? 2 : 0;
    auto I = [&](int m, int k) -> S {
      return hi ? ppm_ip(aR[m], da[m], a6[m], sg[k]) : ppm_im(aL[m], da[m], a6[m], sg[k]);
    };
    auto Ib = [&](int m, int k, S b) {
      if (hi) ppm_ip_vjp(da[m], a6[m], sg[k], b, aRb[m], dab[m], a6b[m], sgb[k]);
      else ppm_im_vjp(da[m], a6[m], sg[k], b, aLb[m], dab[m], a6b[m], sgb[k]);
    };
    S ref[5];
    for (int i = 0; i < 3; ++i) ref[fm[i]] = I(fm[i], kref);
    const bool b1 = hi ? (lam[0] > zero) : (lam[0] < zero);
    const bool b2 = hi ? (lam[1] > zero) : (lam[1] < zero);
    const bool b3 = hi ? (lam[2] > zero) : (lam[2] < zero);
    S a1 = zero, a2 = zero, a3 = zero;
    S dp1 = zero, du1 = zero, dr2 = zero, dp2 = zero, dp3 = zero, du3 = zero;
    if (b1) { dp1 = ref[4] - I(4, 0); du1 = ref[mn] - I(mn, 0); a1 = (dp1 - rc * du1) * hic2; }
    if (b2) { dr2 = ref[0] - I(0, 1); dp2 = ref[4] - I(4, 1); a2 = dr2 - dp2 * ic2; }
    if (b3) { dp3 = ref[4] - I(4, 2); du3 = ref[mn] - I(mn, 2); a3 = (dp3 + rc * du3) * hic2; }
    // edge values (floors frozen; gravity is a constant shift)
    const S q0 = ref[0] - ((a1 + a3) + a2);
    const S q4 = ref[4] - c2 * (a1 + a3);
    const S* qb = hi ? qpb : qmb;
    const S qb0 = (q0 < G.small_dens) ? zero : qb[0];
    const S qb4 = (q4 < G.small_pres) ? zero : qb[4];
    S refb[5];
    for (int i = 0; i < 3; ++i) refb[fm[i]] = zero;
    S a1b = zero, a2b = zero, a3b = zero;
    refb[0] += qb0; a1b -= qb0; a3b -= qb0; a2b -= qb0;
    refb[mn] += qb[mn]; corb += qb[mn] * (a1 - a3); a1b += qb[mn] * cor; a3b -= qb[mn] * cor;
    refb[4] += qb4; c2b -= qb4 * (a1 + a3); a1b -= qb4 * c2; a3b -= qb4 * c2;
    if (b3) {
      const S dp3b = a3b * hic2, du3b = a3b * hic2 * rc;
      rcb += a3b * hic2 * du3;
      hic2b += a3b * (dp3 + rc * du3);
      refb[4] += dp3b; Ib(4, 2, -dp3b);
      refb[mn] += du3b; Ib(mn, 2, -du3b);
    }
    if (b2) {
      const S dr2b = a2b, dp2b = -a2b * ic2;
      ic2b -= a2b * dp2;
      refb[0] += dr2b; Ib(0, 1, -dr2b);
      refb[4] += dp2b; Ib(4, 1, -dp2b);
    }
    if (b1) {
      const S dp1b = a1b * hic2, du1b = -a1b * hic2 * rc;
      rcb -= a1b * hic2 * du1;
      hic2b += a1b * (dp1 - rc * du1);
      refb[4] += dp1b; Ib(4, 0, -dp1b);
      refb[mn] += du1b; Ib(mn, 0, -du1b);
    }
    for (int i = 0; i < 3; ++i) Ib(fm[i], kref, refb[fm[i]]);
    for (int k = 0; k < 3; ++k) {
      const S lk = hi ? lam[k] : -lam[k];
      if (!(lk < zero)) lamb[k] += (hi ? sgb[k] : -sgb[k]) * dtdx;
    }
  }
  unb += lamb[0] + lamb[1] + lamb[2];
  cb += lamb[2] - lamb[0];
  ic2b += HALF * hic2b;
  c2b -= ic2b * ic2 * ic2;
  cb += TWO * c * c2b;
  rb += rcb * c;
  cb += rcb * r;
  const S ir = qdiv(ONE, r);
  cb += corb * ir;
  rb -= corb * cor * ir;
  for (int i = 0; i < 3; ++i) { aRb[fm[i]] += dab[fm[i]]; aLb[fm[i]] -= dab[fm[i]]; }
}

// Reverse of trace_zone<d> for one transverse velocity field with parabola
// (aL, aR, a6): edge adjoints qpb, qmb -> aLb, aRb, a6b; the wave-speed
// adjoints go to lamb (to be added by the coupled fields' reverse).
template <class S>
PPM_HD void trace_transverse_vjp(S aL, S aR, S a6, S un, S c, S dtdx, S qpb, S qmb, S& aLb, S& aRb, S& a6b,
                                 S lamb[3]) {
  const S da = aR - aL;
  S dab = S(0);
  const S lam[3] = {un - c, un, un + c};
  const S zero = S(0);
  for (int side = 0; side < 2; ++side) {
    const bool hi = side == 0;
    const int kref = hi ? 2 : 0;
    S sg[3], sgb[3] = {zero, zero, zero};
    for (int k = 0; k < 3; ++k) sg[k] = smax(hi ? lam[k] : -lam[k], zero) * dtdx;
    const bool b2 = hi ? (lam[1] > zero) : (lam[1] < zero);
    const S qb = hi ? qpb : qmb;
    // q = ref - at, at = ref - I(wave 2) where that wave moves toward the edge
    S refb = qb;
    if (b2) {
      const S atb = -qb;
      refb += atb;
      if (hi) ppm_ip_vjp(da, a6, sg[1], -atb, aRb, dab, a6b, sgb[1]);
      else ppm_im_vjp(da, a6, sg[1], -atb, aLb, dab, a6b, sgb[1]);
    }
    if (hi) ppm_ip_vjp(da, a6, sg[kref], refb, aRb, dab, a6b, sgb[kref]);
    else ppm_im_vjp(da, a6, sg[kref], refb, aLb, dab, a6b, sgb[kref]);
    for (int k = 0; k < 3; ++k) {
      const S lk = hi ? lam[k] : -lam[k];
      if (!(lk < zero)) lamb[k] += (hi ? sgb[k] : -sgb[k]) * dtdx;
    }
  }
  aRb += dab;
  aLb -= dab;
}

}  // namespace ppm
