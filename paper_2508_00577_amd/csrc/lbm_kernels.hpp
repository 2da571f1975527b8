// HIP kernels of one lattice: initialisation, pulled moments, the fused
// stencil + collision step, readout, FP64 reductions and region means.
//
// One time step (eq. pre_LBM), in its two-pass form:
//   k_moments  pull f, g and form rho, j = sum c f, e = sum g into a moment
//              field (the sums of eq. u_shift, eq. T_shift);
//   k_collide  stage rho (tile + 3 halo) in LDS, build lap rho, the force
//              F = a grad(rho^2) + kappa rho grad(lap rho) (eq. EVforce1 with
//              eq. P0E), the half-step fields u, RT, theta = RT/(1 - b rho) on
//              tile + 1, the corrections Phi_aa, Phi', q' (eq. correction_u,
//              correction_gamma, correction_q) and the shifted state (eq.
//              def_ustar) on the tile, then per cell pull f, g again, evaluate
//              the equilibria (eq. feq, f_star, geq, gstar, g_corr), relax and
//              store.
// The one-pass steps need no k_moments launch: in D3Q27 the z-marching
// collision pushes the next step's moments (k_collide_zm<..., PUSH> with
// k_push_fixup); in D2Q9 the collision sums its halo's moments from the
// pulled populations (collide_block<..., FUSED>).
#pragma once

#include <type_traits>

#include "lbm_device.hpp"

namespace evlbm {

template <int S>
using StoreT = typename Codec<S>::T;
template <int S>
using RealT = typename Codec<S>::R;

// -------------------------------------------------------------- k_init

// f = f^eq(rho, u, theta), g = g^eq(u, RT) with theta = P_E/rho = RT Z(rho)
// (eq. feq, eq. geq); inputs in FP64, u may be null (rest).
template <int D, int S>
__global__ void __launch_bounds__(256) k_init(const double *__restrict__ rho0, const double *__restrict__ u0,
                                              const double *__restrict__ T0, StoreT<S> *__restrict__ pop,
                                              StepParams<RealT<S>> p)
{
    using R = RealT<S>;
    constexpr int Q = Lat<D>::Q;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= p.N) return;
    const double rho = rho0[cell];
    const double RT = (double)p.Rgas * T0[cell];
    double Z = 0.0;  // the fields were validated: inside the closure's range
    enskog_z64(p.eos, (double)p.b, rho, &Z);
    const double theta = RT * Z;
    double u[3] = {0.0, 0.0, 0.0};
    if (u0)
        for (int a = 0; a < D; ++a) u[a] = u0[a * p.N + cell];
    double fe[3][3], xe[3][3];
    for (int a = 0; a < 3; ++a) {
        if (a < D) {
            psi3<double>(u[a], theta + u[a] * u[a], fe[a]);
            chi3<double>(u[a], theta, xe[a]);
        } else {
            fe[a][0] = fe[a][2] = 0.0;
            fe[a][1] = 1.0;
            xe[a][0] = xe[a][1] = xe[a][2] = 0.0;
        }
    }
    const double h = 1.5 * RT;
    const float4 rs = ref_state_at<S>(p, cell);
    const RefInv<R> inv = ref_inv_of<S, R>(rs);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int kx = cx_of(i) + 1, ky = cy_of(i) + 1, kz = cz_d<D>(i) + 1;
        const double f = rho * fe[0][kx] * fe[1][ky] * fe[2][kz];
        const double g = rho * ((h * fe[0][kx] + xe[0][kx]) * fe[1][ky] * fe[2][kz] +
                                fe[0][kx] * (xe[1][ky] * fe[2][kz] + fe[1][ky] * xe[2][kz]));
        pop[(long)i * p.ds + cell] = Codec<S>::enc((R)f, ref_enc<D, S>(i, rs, inv));
        pop[(long)(Q + i) * p.ds + cell] = Codec<S>::enc((R)g, ref_enc<D, S>(Q + i, rs, inv));
    }
}

// ------------------------------------------------------------ k_moments

// Raw moments of the pulled populations fh_i(x) = f_i(x - c_i), gh_i
// likewise, of cell (x, y, z) (the density and the sums of eq. u_shift and
// eq. T_shift before their force terms): out = {rho, jx, jy, jz, e}, each
// summed in direction order.  WITH_F: rho and j (from f); WITH_G: e (from g).
template <int D, int S, bool WITH_F = true, bool WITH_G = true>
__device__ inline void pulled_moments(const StoreT<S> *__restrict__ pop, const StepParams<RealT<S>> &p, int x, int y,
                                      int z, RealT<S> out[5])
{
    using R = RealT<S>;
    constexpr int Q = Lat<D>::Q;
    const PullOffsets o = pull_offsets<D, (int)sizeof(StoreT<S>)>(p.nx, p.ny, p.nz, x, y, z);
    R rho = R(0), jx = R(0), jy = R(0), jz = R(0), e = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const unsigned s = o.ox[cx_of(i) + 1] + o.oy[cy_of(i) + 1] + o.oz[cz_d<D>(i) + 1];
        if constexpr (WITH_F) {
            const R f = Codec<S>::dec(ld_at(pop + (long)i * p.ds, s), ref_at_b<D, S>(p, i, s));
            rho += f;
            if (cx_of(i) == 1) jx += f;
            if (cx_of(i) == -1) jx -= f;
            if (cy_of(i) == 1) jy += f;
            if (cy_of(i) == -1) jy -= f;
            if (cz_d<D>(i) == 1) jz += f;
            if (cz_d<D>(i) == -1) jz -= f;
        }
        if constexpr (WITH_G) {
            const R g = Codec<S>::dec(ld_at(pop + (long)(Q + i) * p.ds, s), ref_at_b<D, S>(p, Q + i, s));
            e += g;
        }
    }
    out[0] = rho;
    out[1] = jx;
    out[2] = jy;
    out[3] = jz;
    out[4] = e;
}

// m[0] = rho, m[1..D] = j, m[D+1] = e of the pulled populations
// fh_i(x) = f_i(x - c_i).  Grid (ceil(nx/bx), ny, nz), block (bx).
template <int D, int S>
__device__ inline void moments_at(const StoreT<S> *__restrict__ pop, RealT<S> *__restrict__ m,
                                  const StepParams<RealT<S>> &p, int x, int y, int z)
{
    using R = RealT<S>;
    R mo[5];
    pulled_moments<D, S>(pop, p, x, y, z, mo);
    const unsigned c = ((unsigned)x + (unsigned)p.nx * ((unsigned)y + (unsigned)p.ny * (unsigned)z)) * (unsigned)sizeof(R);
    st_at(m, c, mo[0]);
    st_at(m + p.N, c, mo[1]);
    st_at(m + 2 * p.N, c, mo[2]);
    if (D == 3) st_at(m + 3 * p.N, c, mo[3]);
    st_at(m + (D + 1) * p.N, c, mo[4]);
}

template <int D, int S>
__global__ void __launch_bounds__(256) k_moments(const StoreT<S> *__restrict__ pop, RealT<S> *__restrict__ m,
                                                 StepParams<RealT<S>> p)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= p.nx) return;
    moments_at<D, S>(pop, m, p, x, blockIdx.y, blockIdx.z);
}

// Raw stored values of the pulled populations fh_i(x) = f_i(x - c_i), gh_i
// likewise, of the cell whose pull sources are o, through the population
// accessor (PtrPops or BufPops).  Issued as independent loads so a caller can
// overlap them with other work before decoding.
template <int D, int S, class A>
__device__ inline void pull_pops(const A &pops, const PullOffsets &o, StoreT<S> fr[], StoreT<S> gr[])
{
    constexpr int Q = Lat<D>::Q;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const unsigned s = o.ox[cx_of(i) + 1] + o.oy[cy_of(i) + 1] + o.oz[cz_d<D>(i) + 1];
        fr[i] = pops.ld(i, s);
        gr[i] = pops.ld(Q + i, s);
    }
}

// Error-free sums for the conservation closure, in the arithmetic type.
// Knuth's TwoSum (TAOCP vol. 2, 4.2.2): s = fl(a + b) and e with s + e = a + b
// exactly, for any a, b (6 operations).
template <typename R>
__device__ inline void two_sum(R a, R b, R &s, R &e)
{
    s = a + b;
    const R bv = s - a;
    e = (a - (s - bv)) + (b - bv);
}

// A sum carried as hi + lo.  add() is Dekker's Fast2Sum (1971): for
// |hi| >= |x|, s = fl(hi + x) and x - (s - hi) is the exact rounding error of
// s, which lo collects (3 operations and one add).  The collision starts hi
// at the cell's rest population, the largest population whenever
// theta + u_a^2 + |u_a| < 2 (1 - theta - u_a^2) on every axis (all the states
// of these workloads), and adds and subtracts single populations, so the
// error terms are exact; lo rounds only sums of errors that are each below
// half an ulp of hi, i.e. the pair carries ~2^-48 of the cell's mass.
template <typename R>
struct Compensated {
    R hi, lo;
    __device__ inline void add(R x)
    {
        const R s = hi + x;
        lo += x - (s - hi);
        hi = s;
    }
    // exact product a b = p + e (e from a fused multiply-add) added in
    __device__ inline void add_product(R a, R b)
    {
        const R pr = a * b;
        R e;
        if constexpr (sizeof(R) == 4)
            e = __builtin_fmaf(a, b, -pr);
        else
            e = __builtin_fma(a, b, -pr);
        add(pr);
        lo += e;
    }
};

// Store the rest direction r and the opposite pair a, b of a cell so that
// their three stored values sum to the compensated total t up to the pair's
// own rounding: r gets t - na - nb, the pair its updates na, nb plus half of
// the rest's rounding residual each (b also absorbs a's rounding).  The two
// differences of nearby values that carry the balance (t - r, pair - a) are
// formed exactly with TwoSum.  The values the three stored words decode to
// are returned in out (r, a, b).
template <int S, class A>
__device__ inline void close_three(const A &pops, unsigned cell, int r, int a, int b, Compensated<RealT<S>> t,
                                   RealT<S> na, RealT<S> nb, Ref<RealT<S>> qr, Ref<RealT<S>> qa, Ref<RealT<S>> qb,
                                   RealT<S> out[3])
{
    using R = RealT<S>;
    const StoreT<S> vr = Codec<S>::enc(((t.hi - na) - nb) + t.lo, qr);
    out[0] = Codec<S>::dec(vr, qr);
    R ph, pl;  // what a + b must carry: t - out[0] = ph + pl
    two_sum(t.hi, -out[0], ph, pl);
    pl += t.lo;
    const R half = R(0.5) * (((ph - na) - nb) + pl);  // half the rest's residual
    const StoreT<S> va = Codec<S>::enc(na + half, qa);
    out[1] = Codec<S>::dec(va, qa);
    R bh, bl;  // what b must carry: ph + pl - out[1]
    two_sum(ph, -out[1], bh, bl);
    const StoreT<S> vb = Codec<S>::enc(bh + (bl + pl), qb);
    out[2] = Codec<S>::dec(vb, qb);
    pops.st(r, cell, vr);
    pops.st(a, cell, va);
    pops.st(b, cell, vb);
}

// Receiver of the values a collision stores, as they decode (the next step
// pulls exactly these): sink(i, f_i, g_i) once per direction.
struct NoSink {
    template <typename R>
    __device__ inline void operator()(int, R, R) const {}
};

// Equilibria (eq. feq, f_star, geq, gstar with eq. g_corr), shifted state
// (eq. def_ustar with Qtilde = 0) and the update eq. pre_LBM for one cell,
// f with beta and g with beta_g (Prandtl number Pr = tau/tau_g; Pr = 1 is the
// paper's scheme).  For Pr != 1 (the VPR kernels) g also relaxes its
// viscous-heating flux with f's beta through a quasi-equilibrium term
// qe dg, qe = 2 (beta_g - beta), dg_i = (1/2) c_i . (u . Pi^neq) on the axis
// directions, Pi^neq = sum_i c_i c_i (fh_i - f^eq_i): the Fourier flux then
// scales with tau_g and the viscous heating with tau (k = (5/2) R mu/Pr),
// mass and energy unchanged;
// from its pulled populations (raw stored values fr, gr of pull_pops) into
// the destination of the accessor at the cell itself (o.ox[1] + o.oy[1] +
// o.oz[1]).  zf = Z(rho) = P_E/(rho R T) (enskog).  Every stored direction is also handed
// to sink, decoded.
template <int D, int S, class A, class Sink = NoSink, bool VPR = false>
__device__ inline void collide_pulled(const StoreT<S> fr[], const StoreT<S> gr[], const A &pops,
                                      const StepParams<RealT<S>> &p, const PullOffsets &o, RealT<S> rho,
                                      RealT<S> inv_rho, RealT<S> K, RealT<S> zf, RealT<S> theta,
                                      const RealT<S> u[3], const RealT<S> F[3], const RealT<S> Phi[3],
                                      const RealT<S> qp[3], Sink sink = Sink())
{
    using R = RealT<S>;
    constexpr int Q = Lat<D>::Q;
    // shifted state (eq. def_ustar, Qtilde = 0)
    R us[3], F2 = R(0);
    for (int a = 0; a < 3; ++a) {
        us[a] = u[a] + p.lambda * F[a] * inv_rho;
        F2 += F[a] * F[a];
    }
    // (3/2) RT* = (3/2) RT - lambda^2 |F|^2/(2 rho^2)
    const R hS = K - R(0.5) * p.lambda * p.lambda * F2 * inv_rho * inv_rho;
    const R RTs = hS * (R(2) / R(3));
    const R thetas = RTs * zf;

    // per-axis factors: fe (f^eq and g^eq), fs (f*), gs (g*), chi for g^eq, g*
    R fe[3][3], fs[3][3], gs[3][3], xe[3][3], xs[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a < D) {
            psi3<R>(u[a], theta + u[a] * u[a], fe[a]);
            psi3<R>(us[a], theta + us[a] * us[a] + p.lambda * Phi[a] * inv_rho, fs[a]);
            psi3<R>(us[a], thetas + us[a] * us[a], gs[a]);
            chi3<R>(u[a], theta, xe[a]);
            chi3<R>(us[a], thetas, xs[a]);
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                fe[a][k] = fs[a][k] = gs[a][k] = (k == 1) ? R(1) : R(0);
                xe[a][k] = xs[a][k] = R(0);
            }
        }
    }
    const R hE = K;
    const R omb = R(1) - p.two_beta;
    const R c_eq = p.two_beta - p.wstar;
    const R omb_g = R(1) - p.two_beta_g;
    const R c_eq_g = p.two_beta_g - p.wstar_g;
    const unsigned cell = o.ox[1] + o.oy[1] + o.oz[1];
    // u . Pi^neq of the pulled f (quasi-equilibrium flux, Pr != 1 only)
    R upi[3] = {R(0), R(0), R(0)};
    if constexpr (VPR) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int kx = cx_of(i) + 1, ky = cy_of(i) + 1, kz = cz_d<D>(i) + 1;
            const unsigned s = o.ox[kx] + o.oy[ky] + o.oz[kz];
            const R d = Codec<S>::dec(fr[i], ref_at_b<D, S>(p, i, s)) - rho * fe[0][kx] * fe[1][ky] * fe[2][kz];
            const R cu = R(cx_of(i)) * u[0] + R(cy_of(i)) * u[1] + R(cz_d<D>(i)) * u[2];
            upi[0] += R(cx_of(i)) * cu * d;
            upi[1] += R(cy_of(i)) * cu * d;
            upi[2] += R(cz_d<D>(i)) * cu * d;
        }
    }

    // The collision conserves mass and energy exactly: sum f_new = sum fh and
    // sum g_new = sum gh + u.F (eq. pre_LBM with eq. u_shift, T_shift and
    // Qtilde = 0).  Three directions are stored last, after the compensated
    // sums (Compensated: error-free in the arithmetic type) of the incoming
    // values less the values actually stored in the others, with u.F added as
    // exact products: the rest direction takes the remainder less the updates of the
    // two all-diagonal directions c = +-(1, 1[, 1]), and that pair (the
    // smallest populations, ~ (theta/2)^D rho) shares what the rounded rest
    // value leaves, half each, the second member taking the first's rounding
    // too.  The balance then holds to half an ulp of the pair, and the pair's
    // opposite velocities keep the residual out of the momentum.  The rest
    // direction alone is not enough: near a steady state a cell rounds the
    // same way every step, so its rounding accumulates coherently into a mass
    // and energy drift.
    constexpr int REST = (Q - 1) / 2;
    constexpr int SA = Q - 1, SB = 0;  // c = (+1, +1[, +1]) and (-1, -1[, -1])
    const float4 rsc = ref_state_at_b<S>(p, cell);  // the cell's own reference state
    const RefInv<R> invc = ref_inv_of<S, R>(rsc);
    const R fh_rest = Codec<S>::dec(fr[REST], ref_enc<D, S>(REST, rsc, invc));
    const R gh_rest = Codec<S>::dec(gr[REST], ref_enc<D, S>(Q + REST, rsc, invc));
    Compensated<R> mass{fh_rest, R(0)}, energy{gh_rest, R(0)};
    R fn_a = R(0), gn_a = R(0), fn_b = R(0), gn_b = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (i == REST) continue;
        const int kx = cx_of(i) + 1, ky = cy_of(i) + 1, kz = cz_d<D>(i) + 1;
        const unsigned s = o.ox[kx] + o.oy[ky] + o.oz[kz];
        const R fh = Codec<S>::dec(fr[i], ref_at_b<D, S>(p, i, s));
        const R gh = Codec<S>::dec(gr[i], ref_at_b<D, S>(p, Q + i, s));
        const R Pyz_e = fe[1][ky] * fe[2][kz];
        const R feq = rho * fe[0][kx] * Pyz_e;
        const R fst = rho * fs[0][kx] * (fs[1][ky] * fs[2][kz]);
        const R geq = rho * ((hE * fe[0][kx] + xe[0][kx]) * Pyz_e +
                             fe[0][kx] * (xe[1][ky] * fe[2][kz] + fe[1][ky] * xe[2][kz]));
        R gst = rho * ((hS * gs[0][kx] + xs[0][kx]) * (gs[1][ky] * gs[2][kz]) +
                       gs[0][kx] * (xs[1][ky] * gs[2][kz] + gs[1][ky] * xs[2][kz]));
        R gqe = R(0);
        if (cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_d<D>(i) * cz_d<D>(i) == 1) {
            gst += R(0.5) * (R(cx_of(i)) * qp[0] + R(cy_of(i)) * qp[1] + R(cz_d<D>(i)) * qp[2]);
            if (VPR) gqe = R(0.5) * p.qe * (R(cx_of(i)) * upi[0] + R(cy_of(i)) * upi[1] + R(cz_d<D>(i)) * upi[2]);
        }
        // eq. pre_LBM: f + 2 beta (f^eq - f) + (dt/lambda)(1 - beta)(f* - f^eq),
        // g the same with beta_g (plus the quasi-equilibrium term for Pr != 1)
        const R fn = omb * fh + c_eq * feq + p.wstar * fst;
        const R gn = VPR ? omb_g * gh + c_eq_g * geq + p.wstar_g * gst + gqe : omb_g * gh + c_eq_g * geq + p.wstar_g * gst;
        mass.add(fh);
        energy.add(gh);
        if (i == SA) {
            fn_a = fn;
            gn_a = gn;
            continue;
        }
        if (i == SB) {
            fn_b = fn;
            gn_b = gn;
            continue;
        }
        const Ref<R> rf = ref_enc<D, S>(i, rsc, invc), rg = ref_enc<D, S>(Q + i, rsc, invc);
        const StoreT<S> fq = Codec<S>::enc(fn, rf);
        const StoreT<S> gq = Codec<S>::enc(gn, rg);
        pops.st(i, cell, fq);
        pops.st(Q + i, cell, gq);
        // FP32 and FP64 storage: keep the stores here.  The scheduler
        // otherwise sinks all 2Q of them to the end, and the next plane's
        // loads, which reuse their source registers, must then wait for every
        // one of them to retire.  (With 16-bit storage the pinned order
        // measured slower.)
        if constexpr (sizeof(StoreT<S>) >= 4) __builtin_amdgcn_sched_barrier(0);
        const R fd = Codec<S>::dec(fq, rf), gd = Codec<S>::dec(gq, rg);
        mass.add(-fd);
        energy.add(-gd);
        sink(i, fd, gd);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) energy.add_product(u[a], F[a]);
    R cf[3], cg[3];
    close_three<S>(pops, cell, REST, SA, SB, mass, fn_a, fn_b, ref_enc<D, S>(REST, rsc, invc),
                   ref_enc<D, S>(SA, rsc, invc), ref_enc<D, S>(SB, rsc, invc), cf);
    close_three<S>(pops, cell, Q + REST, Q + SA, Q + SB, energy, gn_a, gn_b,
                   ref_enc<D, S>(Q + REST, rsc, invc), ref_enc<D, S>(Q + SA, rsc, invc),
                   ref_enc<D, S>(Q + SB, rsc, invc), cg);
    sink(REST, cf[0], cg[0]);
    sink(SA, cf[1], cg[1]);
    sink(SB, cf[2], cg[2]);
}

// Pull and collide one cell (x, y, z) from src into dst.
template <int D, int S, bool VPR = false>
__device__ inline void collide_cell(const StoreT<S> *__restrict__ src, StoreT<S> *__restrict__ dst,
                                    const StepParams<RealT<S>> &p, int x, int y, int z, RealT<S> rho,
                                    RealT<S> inv_rho, RealT<S> K, RealT<S> RT, RealT<S> zf, RealT<S> theta,
                                    const RealT<S> u[3], const RealT<S> F[3], const RealT<S> Phi[3],
                                    const RealT<S> qp[3])
{
    constexpr int Q = Lat<D>::Q;
    (void)RT;
    const PullOffsets o = pull_offsets<D, (int)sizeof(StoreT<S>)>(p.nx, p.ny, p.nz, x, y, z);
    const PtrPops<StoreT<S>> pops{src, dst, p.ds};
    StoreT<S> fr[Q], gr[Q];
    pull_pops<D, S>(pops, o, fr, gr);
    collide_pulled<D, S, PtrPops<StoreT<S>>, NoSink, VPR>(fr, gr, pops, p, o, rho, inv_rho, K, zf, theta, u, F, Phi,
                                                          qp);
}

// ------------------------------------------------------------ k_collide

// Tile of block b (tiles x fastest, then y, then the z chunk; T tiles per
// chunk).  Workgroups are dealt round-robin to the 8 XCDs, each with its own
// L2: XCD j gets the j-th eighth of every chunk, whole rows of tiles, so
// tiles that share halo lines are resident on the same L2 while all XCDs
// stream the same chunk (HBM page locality).  Identity when 8 does not
// divide T; a bijection either way.
__host__ __device__ inline int xcd_tile(int b, int T)
{
    if (T & 7) return b;
    const int per = T >> 3, j = b & 7, k = b >> 3;
    return (k / per) * T + j * per + k % per;
}

template <int D, int BX, int BY, int BZ>
struct TileShape {
    static constexpr int HZ = Lat<D>::HZ;
    static constexpr int R3X = BX + 6, R3Y = BY + 6, R3Z = BZ + 6 * HZ;
    static constexpr int R2X = BX + 4, R2Y = BY + 4, R2Z = BZ + 4 * HZ;
    static constexpr int R1X = BX + 2, R1Y = BY + 2, R1Z = BZ + 2 * HZ;
    static constexpr int N3 = R3X * R3Y * R3Z, N2 = R2X * R2Y * R2Z, N1 = R1X * R1Y * R1Z;
    // fields kept on tile + 1: u (D), M = rho u (u^2 + 3 theta - 1) (D), F (D),
    // theta - RT, K = (3/2) RT
    static constexpr int NF = 3 * D + 2;
    static constexpr int NT = BX * BY * BZ;
};

// One BX x BY x BZ tile of cells with origin (x0, y0, z0); the block's
// threads are (threadIdx.x, threadIdx.y, threadIdx.z).  With FUSED (the
// one-pass D2Q9 step) rho on tile + 3 and j, e on tile + 1 are summed here
// from the pulled populations, in the order of the moment kernel, instead of
// read from m (not used), so the step needs no moment pass: rho and j from
// one pull of f in the rho stage (j kept in LDS for tile + 1), e from a pull
// of g in the field stage.
template <int D, int S, int BX, int BY, int BZ, bool FUSED = false, bool VPR = false>
__device__ inline void collide_block(const StoreT<S> *__restrict__ src, StoreT<S> *__restrict__ dst,
                                     const RealT<S> *__restrict__ m, const StepParams<RealT<S>> &p, int x0, int y0,
                                     int z0)
{
    using R = RealT<S>;
    using TS = TileShape<D, BX, BY, BZ>;
    constexpr int Q = Lat<D>::Q;
    constexpr int HZ = TS::HZ;
    constexpr int F_U = 0, F_M = D, F_F = 2 * D, F_TD = 3 * D, F_K = 3 * D + 1;
    __shared__ R s_rho[TS::N3];
    __shared__ R s_lap[TS::N2];
    __shared__ R s_f1[TS::NF * TS::N1];
    __shared__ R s_j[FUSED ? D : 1][FUSED ? TS::N1 : 1];  // FUSED: j on tile + 1, from the rho stage's pulls

    const int tid = threadIdx.x + BX * (threadIdx.y + BY * threadIdx.z);
    const long N = p.N;

    // rho on the tile + 3 halo (periodic)
    for (int t = tid; t < TS::N3; t += TS::NT) {
        const int lx = t % TS::R3X, ly = (t / TS::R3X) % TS::R3Y, lz = t / (TS::R3X * TS::R3Y);
        const int gx = wrapi(x0 + lx - 3, p.nx), gy = wrapi(y0 + ly - 3, p.ny);
        const int gz = HZ ? wrapi(z0 + lz - 3, p.nz) : 0;
        if constexpr (FUSED) {
            R mo[5];
            pulled_moments<D, S, true, false>(src, p, gx, gy, gz, mo);
            s_rho[t] = mo[0];
            const int l1x = lx - 2, l1y = ly - 2, l1z = lz - 2 * HZ;
            if (l1x >= 0 && l1x < TS::R1X && l1y >= 0 && l1y < TS::R1Y && l1z >= 0 && l1z < TS::R1Z)
                for (int a = 0; a < D; ++a) s_j[a][l1x + TS::R1X * (l1y + TS::R1Y * l1z)] = mo[1 + a];
        } else {
            s_rho[t] = m[(long)gx + (long)p.nx * ((long)gy + (long)p.ny * gz)];
        }
    }
    __syncthreads();

    // lap rho on tile + 2
    for (int t = tid; t < TS::N2; t += TS::NT) {
        const int lx = t % TS::R2X, ly = (t / TS::R2X) % TS::R2Y, lz = t / (TS::R2X * TS::R2Y);
        const int c3 = (lx + 1) + TS::R3X * ((ly + 1) + TS::R3Y * (lz + HZ));
        s_lap[t] = lds_lap<D, R>(s_rho, c3, TS::R3X, TS::R3X * TS::R3Y);
    }
    __syncthreads();

    // force and half-step fields on tile + 1 (eq. EVforce1 under eq. P0E;
    // eq. u_shift, eq. T_shift with Qtilde = 0)
    for (int t = tid; t < TS::N1; t += TS::NT) {
        const int lx = t % TS::R1X, ly = (t / TS::R1X) % TS::R1Y, lz = t / (TS::R1X * TS::R1Y);
        const int c3 = (lx + 2) + TS::R3X * ((ly + 2) + TS::R3Y * (lz + 2 * HZ));
        const int c2 = (lx + 1) + TS::R2X * ((ly + 1) + TS::R2Y * (lz + HZ));
        const R rho = s_rho[c3];
        R F[3];
        F[0] = p.a * lds_grad_sq<D, 0, R>(s_rho, c3, TS::R3X, TS::R3X * TS::R3Y) +
               p.kappa * rho * lds_grad<D, 0, R>(s_lap, c2, TS::R2X, TS::R2X * TS::R2Y);
        F[1] = p.a * lds_grad_sq<D, 1, R>(s_rho, c3, TS::R3X, TS::R3X * TS::R3Y) +
               p.kappa * rho * lds_grad<D, 1, R>(s_lap, c2, TS::R2X, TS::R2X * TS::R2Y);
        F[2] = (D == 3) ? p.a * lds_grad_sq<D, 2, R>(s_rho, c3, TS::R3X, TS::R3X * TS::R3Y) +
                              p.kappa * rho * lds_grad<D, 2, R>(s_lap, c2, TS::R2X, TS::R2X * TS::R2Y)
                        : R(0);
        const int gx = wrapi(x0 + lx - 1, p.nx), gy = wrapi(y0 + ly - 1, p.ny);
        const int gz = HZ ? wrapi(z0 + lz - 1, p.nz) : 0;
        R mj[3], me;
        if constexpr (FUSED) {
            R mo[5];
            pulled_moments<D, S, false, true>(src, p, gx, gy, gz, mo);
            for (int a = 0; a < D; ++a) mj[a] = s_j[a][t];
            me = mo[4];
        } else {
            const long cell = (long)gx + (long)p.nx * ((long)gy + (long)p.ny * gz);
            for (int a = 0; a < D; ++a) mj[a] = m[(a + 1) * N + cell];
            me = m[(D + 1) * N + cell];
        }
        const R ir = rcp(rho);
        R u[3], uF = R(0), u2 = R(0);
        for (int a = 0; a < D; ++a) {
            u[a] = (mj[a] + R(0.5) * F[a]) * ir;
            uF += u[a] * F[a];
            u2 += u[a] * u[a];
        }
        const R rhoE = me + R(0.5) * uF;
        // K = (3/2) RT is kept as such: the energy equilibria need (3/2) RT and
        // a round trip through a rounded 2/3 would bias the energy every step.
        const R K = rhoE * ir - R(0.5) * u2;
        const R RT = K * (R(2) / R(3));
        const R theta = RT * enskog(p.eos, p.b, rho).Z;
        for (int a = 0; a < D; ++a) {
            s_f1[(F_U + a) * TS::N1 + t] = u[a];
            s_f1[(F_M + a) * TS::N1 + t] = rho * u[a] * (u[a] * u[a] + R(3) * theta - R(1));
            s_f1[(F_F + a) * TS::N1 + t] = F[a];
        }
        s_f1[F_TD * TS::N1 + t] = theta - RT;
        s_f1[F_K * TS::N1 + t] = K;
    }
    __syncthreads();

    const int lx = threadIdx.x, ly = threadIdx.y, lz = threadIdx.z;
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    if (x >= p.nx || y >= p.ny || z >= p.nz) return;
    const int c1 = (lx + 1) + TS::R1X * ((ly + 1) + TS::R1Y * (lz + HZ));
    const int c3 = (lx + 3) + TS::R3X * ((ly + 3) + TS::R3Y * (lz + 3 * HZ));
    constexpr int SY = TS::R1X, SZ = TS::R1X * TS::R1Y;

    const R rho = s_rho[c3];
    const R inv_rho = rcp(rho);
    const R K = s_f1[F_K * TS::N1 + c1];  // (3/2) RT
    const R RT = K * (R(2) / R(3));
    const Enskog<R> ez = enskog(p.eos, p.b, rho);
    const R theta = RT * ez.Z;
    const R P0 = rho * theta;
    R u[3] = {R(0), R(0), R(0)}, F[3] = {R(0), R(0), R(0)};
    for (int a = 0; a < D; ++a) {
        u[a] = s_f1[(F_U + a) * TS::N1 + c1];
        F[a] = s_f1[(F_F + a) * TS::N1 + c1];
    }
    // corrections (eq. correction_u, correction_gamma with gamma_0 of eq. gamma
    // for P0 = P_E: 5/3 - gamma_0 = ez.g5; eq. correction_q)
    R divu = lds_grad<D, 0, R>(s_f1 + F_U * TS::N1, c1, SY, SZ) +
             lds_grad<D, 1, R>(s_f1 + (F_U + 1) * TS::N1, c1, SY, SZ);
    if (D == 3) divu += lds_grad<D, 2, R>(s_f1 + (F_U + 2) * TS::N1, c1, SY, SZ);
    const R Phip = P0 * ez.g5 * divu;
    R Phi[3] = {R(0), R(0), R(0)}, qp[3] = {R(0), R(0), R(0)};
    Phi[0] = p.sphi * lds_grad<D, 0, R>(s_f1 + F_M * TS::N1, c1, SY, SZ) + Phip;
    Phi[1] = p.sphi * lds_grad<D, 1, R>(s_f1 + (F_M + 1) * TS::N1, c1, SY, SZ) + Phip;
    qp[0] = p.lambda * (P0 * lds_grad<D, 0, R>(s_f1 + F_TD * TS::N1, c1, SY, SZ) + u[0] * Phip);
    qp[1] = p.lambda * (P0 * lds_grad<D, 1, R>(s_f1 + F_TD * TS::N1, c1, SY, SZ) + u[1] * Phip);
    if (D == 3) {
        Phi[2] = p.sphi * lds_grad<D, 2, R>(s_f1 + (F_M + 2) * TS::N1, c1, SY, SZ) + Phip;
        qp[2] = p.lambda * (P0 * lds_grad<D, 2, R>(s_f1 + F_TD * TS::N1, c1, SY, SZ) + u[2] * Phip);
    }
    collide_cell<D, S, VPR>(src, dst, p, x, y, z, rho, inv_rho, K, RT, ez.Z, theta, u, F, Phi, qp);
}

// One tile per workgroup, nbx x nby x nbz tiles in XCD order (xcd_tile).
template <int D, int S, int BX, int BY, int BZ, bool FUSED = false, bool VPR = false>
__global__ void __launch_bounds__(BX *BY *BZ)
    k_collide(const StoreT<S> *__restrict__ src, StoreT<S> *__restrict__ dst, const RealT<S> *__restrict__ m,
              StepParams<RealT<S>> p, int nbx, int nby, int ntiles)
{
    const int t = xcd_tile(blockIdx.x, ntiles), bxy = t % (nbx * nby);
    collide_block<D, S, BX, BY, BZ, FUSED, VPR>(src, dst, m, p, (bxy % nbx) * BX, (bxy / nbx) * BY,
                                                (t / (nbx * nby)) * BZ);
}

// ------------------------------------------------------- k_collide_zm (3D)

// D3Q27 variant that marches along z: a workgroup owns a TX x TY column of
// cells and walks a chunk of ZC planes, keeping the per-plane inputs of the
// stencil chain in LDS ring buffers, so the radius-3 halo is recomputed only
// in x and y.  At iteration k it loads rho of plane k+3 (tile + 3), forms
// lap rho of plane k+2 (tile + 2), the force and half-step fields of plane
// k+1 (tile + 1) and collides plane k.  Ring depths: rho 5 planes (k..k+3 are
// read while a fast wave may already write k+4), lap 3, fields 3; the writes
// of iteration k+1 into slots still read in iteration k happen after that
// iteration's first barrier.
template <int TX, int TY>
struct ZTile {
    static constexpr int R3X = TX + 6, R3Y = TY + 6, N3 = R3X * R3Y;
    static constexpr int R2X = TX + 4, R2Y = TY + 4, N2 = R2X * R2Y;
    static constexpr int R1X = TX + 2, R1Y = TY + 2, N1 = R1X * R1Y;
    static constexpr int NT = TX * TY;
    static constexpr int NRHO = 5, NLAP = 3, NFLD = 3;  // ring depths (planes)
    static constexpr int NF = 7;  // u (3), M (3), theta - RT
};

// Isotropic derivative along axis A at in-plane offset c of three planes
// (below, centre, above) with row stride sy.
template <int A, typename R>
__device__ inline R ring_grad(const R *pm, const R *p0, const R *pp, int c, int sy)
{
    const R *pl[3] = {pm, p0, pp};
    R acc = R(0);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int ca = (A == 0) ? dx : (A == 1) ? dy : dz;
                if (ca == 0) continue;
                const R w = R(3) * w1<R>(dx) * w1<R>(dy) * w1<R>(dz) * R(ca);
                acc += w * pl[dz + 1][c + dx + dy * sy];
            }
    return acc;
}

template <int A, typename R>
__device__ inline R ring_grad_sq(const R *pm, const R *p0, const R *pp, int c, int sy)
{
    const R *pl[3] = {pm, p0, pp};
    R acc = R(0);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int ca = (A == 0) ? dx : (A == 1) ? dy : dz;
                if (ca == 0) continue;
                const R w = R(3) * w1<R>(dx) * w1<R>(dy) * w1<R>(dz) * R(ca);
                const R v = pl[dz + 1][c + dx + dy * sy];
                acc += w * (v * v);
            }
    return acc;
}

template <typename R>
__device__ inline R ring_lap(const R *pm, const R *p0, const R *pp, int c, int sy)
{
    const R *pl[3] = {pm, p0, pp};
    const R centre = p0[c];
    R acc = R(0);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const R w = R(6) * w1<R>(dx) * w1<R>(dy) * w1<R>(dz);
                acc += w * (pl[dz + 1][c + dx + dy * sy] - centre);
            }
    return acc;
}

__device__ inline int ring_slot(int k, int n) { return (k + 8 * n) % n; }

// Moments of the next step pushed by the collision (one-pass step).  The
// next step's rho, j and e of a cell are sums over the values stored at its
// 27 pull sources (the left-hand side of eq. pre_LBM).  A tile chunk
// (W x H columns, Zc planes from z0) adds up, per target cell, the part of
// that sum coming from its own cells.  Targets inside the chunk receive it in
// the moment field directly; the targets around it (tile + 1 in x, y and z)
// receive it in the chunk's shell of partial sums, which a fix-up pass adds
// to the owners of those cells.  Shell slots of one moment (SIZE, a multiple
// of 32 values, so that every moment and chunk starts on a 128-byte line):
//   plane lz in [0, Zc), PLANE slots (a multiple of 32): the rows ly = -1 and
//     ly = H with lx in [0, W) (each starts on a line when TX is a multiple
//     of 32), then the columns and corners lx = -1 and lx = W with ly in
//     [-1, H] (together on one line for a 64 x 4 tile)
//   planes lz = -1 and lz = Zc: the whole tile + 1 face, FACE slots each.
// In LDS the collision keeps a plane's ring targets at ring(lx, ly, H), RING
// slots: rows with their corners, then columns.
template <int TX, int TY, int ZC>
struct Shell {
    static constexpr int RING = 2 * (TX + 2) + 2 * TY;
    static constexpr int PLANE = (2 * TX + 2 * (TY + 2) + 31) / 32 * 32;
    static constexpr int FACE = (TX + 2) * (TY + 2);
    static constexpr int SIZE = (ZC * PLANE + 2 * FACE + 31) / 32 * 32;
    __host__ __device__ static int ring(int lx, int ly, int H)
    {
        if (ly < 0) return lx + 1;
        if (ly >= H) return (TX + 2) + lx + 1;
        return 2 * (TX + 2) + (lx < 0 ? ly : TY + ly);
    }
    __host__ __device__ static int face(int lx, int ly) { return (lx + 1) + (TX + 2) * (ly + 1); }
    __host__ __device__ static int slot(int lx, int ly, int lz, int W, int H, int Zc)
    {
        if (lz < 0) return ZC * PLANE + face(lx, ly);
        if (lz >= Zc) return ZC * PLANE + FACE + face(lx, ly);
        if (lx < 0 || lx >= W) return lz * PLANE + 2 * TX + (lx < 0 ? 0 : TY + 2) + ly + 1;
        return lz * PLANE + (ly < 0 ? 0 : TX) + lx;
    }
};

// Value of the lane one to the left (right) in the same tile row, 0 at the
// row's end: the in-row shift of a population with c_x = +1 (-1).  A 64-wide
// row is one wavefront: a DPP whole-wave shift (wave_shr:1 / wave_shl:1 with
// bound_ctrl, so the vacated lane reads 0); narrower rows use a permute.
template <int CTRL>
__device__ inline float dpp_shift(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ inline double dpp_shift(double v)
{
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_mov_dpp(w.x, CTRL, 0xf, 0xf, true),
                                                __builtin_amdgcn_mov_dpp(w.y, CTRL, 0xf, 0xf, true)));
}
template <int TX, typename R>
__device__ inline R from_left(R v, int tx)
{
    if constexpr (TX == 64) return dpp_shift<0x138>(v);  // wave_shr:1, lane t <- t - 1
    const R w = __shfl_up(v, 1, TX);
    return tx == 0 ? R(0) : w;
}
template <int TX, typename R>
__device__ inline R from_right(R v, int tx)
{
    if constexpr (TX == 64) return dpp_shift<0x130>(v);  // wave_shl:1, lane t <- t + 1
    const R w = __shfl_down(v, 1, TX);
    return tx == TX - 1 ? R(0) : w;
}

// BUF selects the population accessor: raw buffer resources (BufPops, valid
// while 27 N sizeof(T) < 2^32) or per-direction pointers (PtrPops).  PUSH
// also writes the next step's moments: the chunk's own part into m_next,
// the rest into its shell (slots of Shell, 5 moments per tile, tiles in
// their natural order); k_push_fixup completes m_next.
template <int S, int TX, int TY, int ZC, bool BUF, bool PUSH, bool VPR = false, int EOSK = -1>
__global__ void __launch_bounds__(TX *TY)
    k_collide_zm(const StoreT<S> *__restrict__ src, StoreT<S> *__restrict__ dst, const RealT<S> *__restrict__ m,
                 StepParams<RealT<S>> p, int nbx, int nby, RealT<S> *__restrict__ m_next,
                 RealT<S> *__restrict__ shell)
{
    using R = RealT<S>;
    using T = StoreT<S>;
    using ZT = ZTile<TX, TY>;
    constexpr int Q = 27;
    constexpr int D = 3;
    constexpr int FU = 0, FM = 3, FTD = 6;
    constexpr int NR3 = (ZT::N3 + ZT::NT - 1) / ZT::NT;  // rho halo values loaded per thread
    constexpr int NR1 = (ZT::N1 + ZT::NT - 1) / ZT::NT;  // field cells per thread
    constexpr unsigned RS = sizeof(R);
    // bytes per moment array; with buffer addressing (27 ds sizeof(T) < 2^32)
    // all five arrays of m lie within 32-bit byte offsets of its base
    const unsigned NB = (unsigned)p.N * RS;
    // rho ring: with PUSH a barrier ends every iteration, so the slot of plane
    // k-1 is free when iteration k writes plane k+3 (4 planes); without it a
    // fast wave may write k+4 while a slow one still reads k (5 planes)
    constexpr int NRHO = PUSH ? 4 : ZT::NRHO;
    __shared__ R s_rho[NRHO][ZT::N3];
    __shared__ R s_lap[ZT::NLAP][ZT::N2];
    __shared__ R s_fld[ZT::NFLD][ZT::NF][ZT::N1];
    // PUSH: in-row sums (Pf = sum f, Jx = sum c_x f, Pg = sum g) per c_z handed
    // to the row above (c_y = +1) and below (c_y = -1); the two end lanes'
    // values leaving the row in x; the ring targets' sums for 3 planes
    using SH = Shell<TX, TY, ZC>;
    constexpr int NXR = PUSH ? TY : 1;
    __shared__ R s_xup[NXR][PUSH ? 9 : 1][PUSH ? TX : 1];  // row ty's parts for row ty + 1 (c_y = +1)
    __shared__ R s_xdn[NXR][PUSH ? 9 : 1][PUSH ? TX : 1];  // row ty's parts for row ty - 1 (c_y = -1)
    __shared__ R s_edge[2][PUSH ? TY : 1][PUSH ? 9 : 1][2];
    __shared__ R s_ring[PUSH ? 3 : 1][PUSH ? 5 : 1][PUSH ? SH::RING : 1];

    // a 64-wide row is one wavefront: its row index is wave-uniform
    const int tx = threadIdx.x, ty = TX == 64 ? __builtin_amdgcn_readfirstlane(threadIdx.y) : threadIdx.y;
    const int tid = tx + TX * ty;
    const int tile = xcd_tile(blockIdx.x, nbx * nby);
    const int x0 = (tile % nbx) * TX, y0 = ((tile / nbx) % nby) * TY;
    const int z0 = (tile / (nbx * nby)) * ZC;
    const int z1 = min(z0 + ZC, p.nz);
    const long N = p.N;
    const unsigned plane = (unsigned)p.nx * (unsigned)p.ny;
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < p.nx && y < p.ny;
    const int W = min(TX, p.nx - x0), H = min(TY, p.ny - y0), Zc = z1 - z0;
    // F and K = (3/2) RT of this thread's own column at planes k (cur) and k+1 (nxt)
    R Fc[3] = {R(0), R(0), R(0)}, Kc = R(0), Fn[3] = {R(0), R(0), R(0)}, Kn = R(0);
    using Pops = typename std::conditional<BUF, BufPops<T, Q>, PtrPops<T>>::type;
    const Pops pops{src, dst, p.ds};

    // in-plane offset (elements) of the halo cells this thread loads
    unsigned o3[NR3];
#pragma unroll
    for (int j = 0; j < NR3; ++j) {
        const int t = min(tid + j * ZT::NT, ZT::N3 - 1);
        const int lx = t % ZT::R3X, ly = t / ZT::R3X;
        o3[j] = (unsigned)wrapi(x0 + lx - 3, p.nx) + (unsigned)p.nx * (unsigned)wrapi(y0 + ly - 3, p.ny);
    }
    // field cells of this thread on tile + 1: interior first (thread tid owns
    // cell (tx, ty)), then the ring: rows 0 and R1Y-1, then columns 0 and R1X-1
    int l1x[NR1], l1y[NR1];
    unsigned o1[NR1];
#pragma unroll
    for (int j = 0; j < NR1; ++j) {
        const int t = min(tid + j * ZT::NT, ZT::N1 - 1);
        int lx, ly;
        if (t < ZT::NT) {
            lx = t % TX + 1;
            ly = t / TX + 1;
        } else {
            const int r = t - ZT::NT;
            if (r < 2 * ZT::R1X) {
                lx = r % ZT::R1X;
                ly = (r < ZT::R1X) ? 0 : ZT::R1Y - 1;
            } else {
                const int q = r - 2 * ZT::R1X;
                lx = (q < TY) ? 0 : ZT::R1X - 1;
                ly = q % TY + 1;
            }
        }
        l1x[j] = lx;
        l1y[j] = ly;
        o1[j] = (unsigned)wrapi(x0 + lx - 1, p.nx) + (unsigned)p.nx * (unsigned)wrapi(y0 + ly - 1, p.ny);
    }

    // Every global load of an iteration is issued up front in straight-line
    // code (no branch around any of them, so the compiler's wait counters stay
    // exact): the populations of plane k, then the moment fields of the next
    // iteration (rho of plane k+4, j and e of plane k+2), so that stage (1)
    // finds its inputs loaded one iteration earlier and stages (1)-(3) run
    // while the populations are in flight.  Halo loads use clamped offsets;
    // threads past a ragged edge pull a valid cell and skip only the stores.
    R rv[NR3], mv[NR1][4], rvn[NR3], mvn[NR1][4];
    auto load_fields = [&](int k, R(&r3)[NR3], R(&r1)[NR1][4]) {
        const unsigned z3 = (unsigned)wrapi(k + 3, p.nz) * plane, z1 = (unsigned)wrapi(k + 1, p.nz) * plane;
#pragma unroll
        for (int j = 0; j < NR3; ++j) r3[j] = ld_at(m, (o3[j] + z3) * RS);
#pragma unroll
        for (int j = 0; j < NR1; ++j)
#pragma unroll
            for (int a = 0; a < 4; ++a) r1[j][a] = BUF ? ld_at(m, (o1[j] + z1) * RS + (a + 1) * NB)
                                                       : ld_at(m + (a + 1) * N, (o1[j] + z1) * RS);
    };
    auto next_fields = [&]() {
#pragma unroll
        for (int j = 0; j < NR3; ++j) rv[j] = rvn[j];
#pragma unroll
        for (int j = 0; j < NR1; ++j)
#pragma unroll
            for (int a = 0; a < 4; ++a) mv[j][a] = mvn[j][a];
    };
    // stages (1)-(3) of iteration k: rho of plane k+3 on tile + 3, lap rho of
    // plane k+2 on tile + 2, force and half-step fields of plane k+1 on tile + 1
    auto stencil_stages = [&](int k, auto &&after_first_barrier) {
        {
            R *dstp = s_rho[ring_slot(k + 3, NRHO)];
#pragma unroll
            for (int j = 0; j < NR3; ++j)
                if (tid + j * ZT::NT < ZT::N3) dstp[tid + j * ZT::NT] = rv[j];
        }
        __syncthreads();
        after_first_barrier();
        {
            const R *a = s_rho[ring_slot(k + 1, NRHO)], *b = s_rho[ring_slot(k + 2, NRHO)],
                    *c = s_rho[ring_slot(k + 3, NRHO)];
            R *dstp = s_lap[ring_slot(k + 2, ZT::NLAP)];
            for (int t = tid; t < ZT::N2; t += ZT::NT) {
                const int lx = t % ZT::R2X, ly = t / ZT::R2X;
                dstp[t] = ring_lap<R>(a, b, c, (lx + 1) + ZT::R3X * (ly + 1), ZT::R3X);
            }
        }
        __syncthreads();
        {
            const R *ra = s_rho[ring_slot(k, NRHO)], *rb = s_rho[ring_slot(k + 1, NRHO)],
                    *rc = s_rho[ring_slot(k + 2, NRHO)];
            const R *la = s_lap[ring_slot(k, ZT::NLAP)], *lb = s_lap[ring_slot(k + 1, ZT::NLAP)],
                    *lc = s_lap[ring_slot(k + 2, ZT::NLAP)];
            R(*fd)[ZT::N1] = s_fld[ring_slot(k + 1, ZT::NFLD)];
#pragma unroll
            for (int j = 0; j < NR1; ++j) {
                if (tid + j * ZT::NT >= ZT::N1) continue;
                const int lx = l1x[j], ly = l1y[j];
                const int c3 = (lx + 2) + ZT::R3X * (ly + 2);
                const int c2 = (lx + 1) + ZT::R2X * (ly + 1);
                const R rho = rb[c3];
                R F[3];
                F[0] = p.a * ring_grad_sq<0, R>(ra, rb, rc, c3, ZT::R3X) + p.kappa * rho * ring_grad<0, R>(la, lb, lc, c2, ZT::R2X);
                F[1] = p.a * ring_grad_sq<1, R>(ra, rb, rc, c3, ZT::R3X) + p.kappa * rho * ring_grad<1, R>(la, lb, lc, c2, ZT::R2X);
                F[2] = p.a * ring_grad_sq<2, R>(ra, rb, rc, c3, ZT::R3X) + p.kappa * rho * ring_grad<2, R>(la, lb, lc, c2, ZT::R2X);
                const R ir = rcp(rho);
                R u[3], uF = R(0), u2 = R(0);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u[a] = (mv[j][a] + R(0.5) * F[a]) * ir;
                    uF += u[a] * F[a];
                    u2 += u[a] * u[a];
                }
                const R K = (mv[j][3] + R(0.5) * uF) * ir - R(0.5) * u2;
                const R RT = K * (R(2) / R(3));
                const R theta = RT * enskog_k<EOSK>(p.eos, p.b, rho).Z;
                const int c1 = lx + ZT::R1X * ly;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    fd[FU + a][c1] = u[a];
                    fd[FM + a][c1] = rho * u[a] * (u[a] * u[a] + R(3) * theta - R(1));
                }
                fd[FTD][c1] = theta - RT;
                if (j == 0) {  // tid < NT: the thread's own column
                    Fn[0] = F[0];
                    Fn[1] = F[1];
                    Fn[2] = F[2];
                    Kn = K;
                }
            }
        }
        __syncthreads();
    };

    // Collision of plane z0 needs the fields of planes z0-1..z0+1, hence lap
    // rho of z0-2..z0+2 and rho of z0-3..z0+3: the pipeline starts 6 planes early.
    load_fields(z0 - 6, rv, mv);
    for (int k = z0 - 6; k < z0; ++k) {
        load_fields(k + 1, rvn, mvn);
        stencil_stages(k, [] {});
        next_fields();
#pragma unroll
        for (int a = 0; a < 3; ++a) Fc[a] = Fn[a];
        Kc = Kn;
    }
    const int xl = min(x, p.nx - 1), yl = min(y, p.ny - 1);

    // PUSH state: the decoded stored values of this cell's collision (zero on
    // lanes past a ragged edge), this thread's own target sums for planes
    // k-1, k, k+1 (rho, jx, jy, jz, e), and the ring targets it owns: the
    // bottom row (tx, -1), the top row (tx, H) and the column targets (-1 or
    // W, c % (H + 2) - 1) on c = tid - TX * TY_COL < 2 (H + 2).  With one row
    // per wave (SPREAD) every row hands both cross-row parts to LDS and the
    // three ring jobs run after the hand-over barrier on waves 1, 2 and 3, so
    // that no wave carries two of them; with several rows per wave the first
    // and last rows commit the ring rows before the barrier from registers
    // (measured faster for the 16 x 8 tile of two waves).
    R vf[Q], vg[Q], acc[3][5];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[j][q] = R(0);
    constexpr bool SPREAD = TX >= 64;
    constexpr int TY_COL = SPREAD ? 3 % TY : (TY > 2 ? 1 : 0);
    static_assert(!PUSH || TX * (TY - TY_COL) >= 2 * (TY + 2), "the column owners must fit in the tile");
    const int ty_bot = SPREAD ? 1 % TY : 0, ty_top = SPREAD ? 2 % TY : H - 1;
    const int col_c = tid - TX * TY_COL;
    const bool col_owner = col_c >= 0 && col_c < 2 * (H + 2);
    const int col_side = col_c >= H + 2 ? 1 : 0, col_ly = col_c - col_side * (H + 2) - 1;
    const int col_lx = col_side ? W : -1;
    R *const shell_t = PUSH ? shell + (long)tile * 5 * SH::SIZE : nullptr;
    if constexpr (PUSH) {
        for (int t = tid; t < 3 * 5 * SH::RING; t += ZT::NT) (&s_ring[0][0][0])[t] = R(0);
        __syncthreads();
    }
    // A ring target (lx, ly) takes source plane kk's parts rc for planes
    // kk-1, kk, kk+1 in one LDS round trip: plane kk-1 is then complete and
    // goes to the shell (its slot cleared for plane kk+2), the other two stay.
    auto ring_commit = [&](int kk, int lx, int ly, const R(&rc)[3][5]) {
        const int ri = SH::ring(lx, ly, H);
        R *r0 = &s_ring[ring_slot(kk - 1, 3)][0][ri], *r1 = &s_ring[ring_slot(kk, 3)][0][ri],
          *r2 = &s_ring[ring_slot(kk + 1, 3)][0][ri];
        R a0[5], a1[5], a2[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            a0[q] = r0[q * SH::RING];
            a1[q] = r1[q * SH::RING];
            a2[q] = r2[q * SH::RING];
        }
        const int sl = SH::slot(lx, ly, kk - 1 - z0, W, H, Zc);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            r0[q * SH::RING] = R(0);
            r1[q * SH::RING] = a1[q] + rc[1][q];
            r2[q * SH::RING] = a2[q] + rc[2][q];
            st_at(shell_t, (unsigned)(q * SH::SIZE + sl) * RS, a0[q] + rc[0][q]);
        }
    };
    // the last two planes of a ring target at the chunk's end
    auto ring_final = [&](int lx, int ly) {
        const int ri = SH::ring(lx, ly, H);
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const int kk = z1 - 1 + d;
            const int sl = SH::slot(lx, ly, kk - z0, W, H, Zc);
#pragma unroll
            for (int q = 0; q < 5; ++q)
                st_at(shell_t, (unsigned)(q * SH::SIZE + sl) * RS, s_ring[ring_slot(kk, 3)][q][ri]);
        }
    };
    // write the finished sums of plane kk of the thread's own target
    auto finish_plane = [&](int kk, const R a[5]) {
        const int lz = kk - z0;
        if (active) {
            if (lz >= 0 && lz < Zc) {
                const unsigned c = ((unsigned)x + (unsigned)p.nx * ((unsigned)y + (unsigned)p.ny * (unsigned)kk)) * RS;
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    if constexpr (BUF)
                        st_at(m_next, c + q * NB, a[q]);
                    else
                        st_at(m_next + q * N, c, a[q]);
                }
            } else {
                const int sl = SH::slot(tx, ty, lz, W, H, Zc);
#pragma unroll
                for (int q = 0; q < 5; ++q) st_at(shell_t, (unsigned)(q * SH::SIZE + sl) * RS, a[q]);
            }
        }
    };
    // push the collided plane k: in-row shifts and sums, the row's own part
    // into acc, the parts for the rows above and below into LDS
    auto push_plane = [&](int k) {
        R rc_dn[3][5], rc_up[3][5];  // without SPREAD: parts for the ring rows below and above the tile
#pragma unroll
        for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
            for (int cy = -1; cy <= 1; ++cy) {
                const int im = 3 * (cy + 1) + 9 * (cz + 1), i0 = im + 1, ip = im + 2;  // c_x = -1, 0, +1
                const R fl = from_left<TX>(vf[ip], tx), fr2 = from_right<TX>(vf[im], tx);
                const R gl = from_left<TX>(vg[ip], tx), gr2 = from_right<TX>(vg[im], tx);
                const R Pf = (fl + vf[i0]) + fr2, Jx = fl - fr2, Pg = (gl + vg[i0]) + gr2;
                const int e = 3 * (cy + 1) + (cz + 1);
                if (!SPREAD && ty < H) {
                    if (tx == 0) {
                        s_edge[0][ty][e][0] = vf[im];
                        s_edge[0][ty][e][1] = vg[im];
                    }
                    if (tx == W - 1) {
                        s_edge[1][ty][e][0] = vf[ip];
                        s_edge[1][ty][e][1] = vg[ip];
                    }
                }
                if (cy == 0) {
                    acc[cz + 1][0] += Pf;
                    acc[cz + 1][1] += Jx;
                    if (cz != 0) acc[cz + 1][3] += cz > 0 ? Pf : -Pf;
                    acc[cz + 1][4] += Pg;
                } else if (cy == 1) {
                    if (SPREAD ? ty < H : ty < H - 1) {
                        s_xup[ty][3 * (cz + 1)][tx] = Pf;
                        s_xup[ty][3 * (cz + 1) + 1][tx] = Jx;
                        s_xup[ty][3 * (cz + 1) + 2][tx] = Pg;
                    }
                    if constexpr (!SPREAD) {
                        rc_up[cz + 1][0] = Pf;
                        rc_up[cz + 1][1] = Jx;
                        rc_up[cz + 1][2] = Pf;
                        rc_up[cz + 1][3] = cz == 0 ? R(0) : cz > 0 ? Pf : -Pf;
                        rc_up[cz + 1][4] = Pg;
                    }
                } else {
                    if ((SPREAD || ty >= 1) && ty < H) {
                        s_xdn[ty][3 * (cz + 1)][tx] = Pf;
                        s_xdn[ty][3 * (cz + 1) + 1][tx] = Jx;
                        s_xdn[ty][3 * (cz + 1) + 2][tx] = Pg;
                    }
                    if constexpr (!SPREAD) {
                        rc_dn[cz + 1][0] = Pf;
                        rc_dn[cz + 1][1] = Jx;
                        rc_dn[cz + 1][2] = -Pf;
                        rc_dn[cz + 1][3] = cz == 0 ? R(0) : cz > 0 ? Pf : -Pf;
                        rc_dn[cz + 1][4] = Pg;
                    }
                }
            }
        // SPREAD: the values leaving the row's end lanes (for the column
        // targets) in one branch after the sums rather than one per group
        // (measured faster for the 64 x 4 tile, slower for the 16 x 8 one)
        if (SPREAD && ty < H && (tx == 0 || tx == W - 1)) {
            const int side = tx == 0 ? 0 : 1;
#pragma unroll
            for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
                for (int cy = -1; cy <= 1; ++cy) {
                    const int im = 3 * (cy + 1) + 9 * (cz + 1), ip = im + 2, e = 3 * (cy + 1) + (cz + 1);
                    s_edge[side][ty][e][0] = side ? vf[ip] : vf[im];
                    s_edge[side][ty][e][1] = side ? vg[ip] : vg[im];
                }
            // a one-column tile's lane is both end lanes: its c_x = +1
            // values leave the row on the right as well
            if (W == 1) {
#pragma unroll
                for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
                    for (int cy = -1; cy <= 1; ++cy) {
                        const int ip = 3 * (cy + 1) + 9 * (cz + 1) + 2, e = 3 * (cy + 1) + (cz + 1);
                        s_edge[1][ty][e][0] = vf[ip];
                        s_edge[1][ty][e][1] = vg[ip];
                    }
            }
        }
        if constexpr (!SPREAD) {
            if (ty == ty_bot && tx < W) ring_commit(k, tx, -1, rc_dn);
            if (ty == ty_top && tx < W) ring_commit(k, tx, H, rc_up);
        }
    };
    // gather the cross-row parts of source plane k (after the barrier that
    // follows its push), then plane k - 1 is complete: write it and rotate
    auto gather_plane = [&](int k) {
        if (active) {
#pragma unroll
            for (int cz = -1; cz <= 1; ++cz) {
                if (ty >= 1) {  // from the row below, c_y = +1
                    const R Pf = s_xup[ty - 1][3 * (cz + 1)][tx];
                    acc[cz + 1][0] += Pf;
                    acc[cz + 1][1] += s_xup[ty - 1][3 * (cz + 1) + 1][tx];
                    acc[cz + 1][2] += Pf;
                    if (cz != 0) acc[cz + 1][3] += cz > 0 ? Pf : -Pf;
                    acc[cz + 1][4] += s_xup[ty - 1][3 * (cz + 1) + 2][tx];
                }
                if (ty + 1 < H) {  // from the row above, c_y = -1
                    const R Pf = s_xdn[ty + 1][3 * (cz + 1)][tx];
                    acc[cz + 1][0] += Pf;
                    acc[cz + 1][1] += s_xdn[ty + 1][3 * (cz + 1) + 1][tx];
                    acc[cz + 1][2] -= Pf;
                    if (cz != 0) acc[cz + 1][3] += cz > 0 ? Pf : -Pf;
                    acc[cz + 1][4] += s_xdn[ty + 1][3 * (cz + 1) + 2][tx];
                }
            }
        }
        // SPREAD: the ring rows below and above the tile, from the first row's
        // parts going down and the last row's going up
        auto commit_row = [&](int ly, const auto &xb, R sy) {
            R rc[3][5];
#pragma unroll
            for (int cz = -1; cz <= 1; ++cz) {
                const R Pf = xb[3 * (cz + 1)][tx];
                rc[cz + 1][0] = Pf;
                rc[cz + 1][1] = xb[3 * (cz + 1) + 1][tx];
                rc[cz + 1][2] = sy * Pf;
                rc[cz + 1][3] = cz == 0 ? R(0) : cz > 0 ? Pf : -Pf;
                rc[cz + 1][4] = xb[3 * (cz + 1) + 2][tx];
            }
            ring_commit(k, tx, ly, rc);
        };
        if constexpr (SPREAD) {
            if (ty == ty_bot && tx < W) commit_row(-1, s_xdn[0], R(-1));
            if (ty == ty_top && tx < W) commit_row(H, s_xup[H - 1], R(1));
        }
        if (col_owner) {  // column and corner targets: values leaving the end lanes
            R rc[3][5];
#pragma unroll
            for (int cz = -1; cz <= 1; ++cz) {
                R f = R(0), fy = R(0), g = R(0);
#pragma unroll
                for (int cy = -1; cy <= 1; ++cy) {
                    const int row = col_ly - cy;
                    if (row >= 0 && row < H) {
                        const R fv = s_edge[col_side][row][3 * (cy + 1) + (cz + 1)][0];
                        f += fv;
                        if (cy != 0) fy += cy > 0 ? fv : -fv;
                        g += s_edge[col_side][row][3 * (cy + 1) + (cz + 1)][1];
                    }
                }
                rc[cz + 1][0] = f;
                rc[cz + 1][1] = col_side ? f : -f;
                rc[cz + 1][2] = fy;
                rc[cz + 1][3] = cz == 0 ? R(0) : cz > 0 ? f : -f;
                rc[cz + 1][4] = g;
            }
            ring_commit(k, col_lx, col_ly, rc);
        }
        finish_plane(k - 1, acc[0]);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            acc[0][q] = acc[1][q];
            acc[1][q] = acc[2][q];
            acc[2][q] = R(0);
        }
    };

    // The populations of plane k+1 are pulled as soon as the collision of
    // plane k has consumed those of plane k, after the next moment fields, so
    // they are in flight through the push, the next iteration's stencil
    // stages and its barriers.  The last iteration pulls plane z1 (a valid
    // plane, not used).
    T fr[Q], gr[Q];
    pull_pops<3, S>(pops, pull_offsets<3, (int)sizeof(T)>(p.nx, p.ny, p.nz, xl, yl, z0), fr, gr);
    for (int k = z0; k < z1; ++k) {
        const PullOffsets po = pull_offsets<3, (int)sizeof(T)>(p.nx, p.ny, p.nz, xl, yl, k);
        stencil_stages(k, [] {});
        // (4) collide plane k
        if (!active) {
            if constexpr (PUSH) {
#pragma unroll
                for (int i = 0; i < Q; ++i) vf[i] = vg[i] = R(0);
            }
        } else {
            const R *fm[ZT::NF], *f0[ZT::NF], *fp[ZT::NF];
#pragma unroll
            for (int q = 0; q < ZT::NF; ++q) {
                fm[q] = s_fld[ring_slot(k - 1, ZT::NFLD)][q];
                f0[q] = s_fld[ring_slot(k, ZT::NFLD)][q];
                fp[q] = s_fld[ring_slot(k + 1, ZT::NFLD)][q];
            }
            const int c1 = (tx + 1) + ZT::R1X * (ty + 1);
            const R rho = s_rho[ring_slot(k, NRHO)][(tx + 3) + ZT::R3X * (ty + 3)];
            const R inv_rho = rcp(rho);
            const R K = Kc;
            const R RT = K * (R(2) / R(3));
            const Enskog<R> ez = enskog_k<EOSK>(p.eos, p.b, rho);
            const R theta = RT * ez.Z;
            const R P0 = rho * theta;
            R u[3], F[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u[a] = f0[FU + a][c1];
                F[a] = Fc[a];
            }
            const R divu = ring_grad<0, R>(fm[FU], f0[FU], fp[FU], c1, ZT::R1X) +
                           ring_grad<1, R>(fm[FU + 1], f0[FU + 1], fp[FU + 1], c1, ZT::R1X) +
                           ring_grad<2, R>(fm[FU + 2], f0[FU + 2], fp[FU + 2], c1, ZT::R1X);
            const R Phip = P0 * ez.g5 * divu;
            R Phi[3], qp[3];
            Phi[0] = p.sphi * ring_grad<0, R>(fm[FM], f0[FM], fp[FM], c1, ZT::R1X) + Phip;
            Phi[1] = p.sphi * ring_grad<1, R>(fm[FM + 1], f0[FM + 1], fp[FM + 1], c1, ZT::R1X) + Phip;
            Phi[2] = p.sphi * ring_grad<2, R>(fm[FM + 2], f0[FM + 2], fp[FM + 2], c1, ZT::R1X) + Phip;
            qp[0] = p.lambda * (P0 * ring_grad<0, R>(fm[FTD], f0[FTD], fp[FTD], c1, ZT::R1X) + u[0] * Phip);
            qp[1] = p.lambda * (P0 * ring_grad<1, R>(fm[FTD], f0[FTD], fp[FTD], c1, ZT::R1X) + u[1] * Phip);
            qp[2] = p.lambda * (P0 * ring_grad<2, R>(fm[FTD], f0[FTD], fp[FTD], c1, ZT::R1X) + u[2] * Phip);
            if constexpr (PUSH) {
                auto push_sink = [&](int i, R f, R g) {
                    vf[i] = f;
                    vg[i] = g;
                };
                collide_pulled<D, S, Pops, decltype(push_sink), VPR>(fr, gr, pops, p, po, rho, inv_rho, K, ez.Z,
                                                                       theta, u, F, Phi, qp, push_sink);
            } else
                collide_pulled<D, S, Pops, NoSink, VPR>(fr, gr, pops, p, po, rho, inv_rho, K, ez.Z, theta, u, F, Phi,
                                                        qp);
        }
        load_fields(k + 1, rvn, mvn);
        pull_pops<3, S>(pops, pull_offsets<3, (int)sizeof(T)>(p.nx, p.ny, p.nz, xl, yl, k + 1), fr, gr);
        if constexpr (PUSH) {
            push_plane(k);
            __syncthreads();
            gather_plane(k);
        }
        next_fields();
        // rotate the column's F, K
#pragma unroll
        for (int a = 0; a < 3; ++a) Fc[a] = Fn[a];
        Kc = Kn;
    }
    if constexpr (PUSH) {
        // planes z1 - 1 (inside the chunk) and z1 (the face above)
        finish_plane(z1 - 1, acc[0]);
        finish_plane(z1, acc[1]);
        if (ty == ty_bot && tx < W) ring_final(tx, -1);
        if (ty == ty_top && tx < W) ring_final(tx, H);
        if (col_owner) ring_final(col_lx, col_ly);
    }
}

// Completes the pushed moments: a cell on a face of its tile chunk gets, in a
// fixed order, the partial sums that the neighbouring chunks left for it in
// their shells.  In each axis the candidates are the own chunk, the one
// before (if the cell is the chunk's first, it lies on that chunk's far side)
// and the one after (if it is the last; on that chunk's near side); a lattice
// one chunk wide is its own neighbour, so periodic wrap needs no special case.
// One workgroup of TX x TY threads per plane of a tile chunk (blockIdx.x the
// chunk in natural order, blockIdx.y the plane), a thread per cell: the cells
// of a chunk's planes are independent, so no wave walks the chunk's planes
// one after another.
template <typename R, int TX, int TY, int ZC>
__global__ void __launch_bounds__(TX *TY) k_push_fixup(R *__restrict__ m, const R *__restrict__ shell, int nx, int ny,
                                                       int nz, int nbx, int nby, int nbz)
{
    using SH = Shell<TX, TY, ZC>;
    const int tile = blockIdx.x, lz = blockIdx.y;
    const int bx = tile % nbx, by = (tile / nbx) % nby, bz = tile / (nbx * nby);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * ZC;
    const int W = min(TX, nx - x0), H = min(TY, ny - y0), Zc = min(ZC, nz - z0);
    const int tx = threadIdx.x, ty = threadIdx.y;
    if (tx >= W || ty >= H || lz >= Zc) return;
    const unsigned N = (unsigned)nx * (unsigned)ny * (unsigned)nz;
    // candidates per axis: tile index offset and the cell's local coordinate in that tile
    int nxc = 1, nyc = 1, txi[3] = {bx, 0, 0}, lxs[3] = {tx, 0, 0}, tyi[3] = {by, 0, 0}, lys[3] = {ty, 0, 0};
    if (tx == 0) {
        const int b2 = bx == 0 ? nbx - 1 : bx - 1;
        txi[nxc] = b2;
        lxs[nxc++] = min(TX, nx - b2 * TX);
    }
    if (tx == W - 1) {
        txi[nxc] = bx == nbx - 1 ? 0 : bx + 1;
        lxs[nxc++] = -1;
    }
    if (ty == 0) {
        const int b2 = by == 0 ? nby - 1 : by - 1;
        tyi[nyc] = b2;
        lys[nyc++] = min(TY, ny - b2 * TY);
    }
    if (ty == H - 1) {
        tyi[nyc] = by == nby - 1 ? 0 : by + 1;
        lys[nyc++] = -1;
    }
    int nzc = 1, tzi[3] = {bz, 0, 0}, lzs[3] = {lz, 0, 0};
    if (lz == 0) {
        const int bzm = bz == 0 ? nbz - 1 : bz - 1;
        tzi[nzc] = bzm;
        lzs[nzc++] = min(ZC, nz - bzm * ZC);
    }
    if (lz == Zc - 1) {
        tzi[nzc] = bz == nbz - 1 ? 0 : bz + 1;
        lzs[nzc++] = -1;
    }
    if (nzc == 1 && nxc == 1 && nyc == 1) return;  // inside the chunk: complete already
    const unsigned cell = (unsigned)(x0 + tx) + (unsigned)nx * ((unsigned)(y0 + ty) + (unsigned)ny * (unsigned)(z0 + lz));
    R sum[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) sum[q] = m[q * (size_t)N + cell];
    for (int kz = 0; kz < nzc; ++kz) {
        const int Zc2 = min(ZC, nz - tzi[kz] * ZC);
        for (int ky = 0; ky < nyc; ++ky) {
            const int H2 = min(TY, ny - tyi[ky] * TY);
            for (int kx = 0; kx < nxc; ++kx) {
                if (kx == 0 && ky == 0 && kz == 0) continue;
                const int W2 = min(TX, nx - txi[kx] * TX);
                const R *sh = shell + (size_t)(txi[kx] + nbx * (tyi[ky] + nby * tzi[kz])) * 5 * SH::SIZE +
                              SH::slot(lxs[kx], lys[ky], lzs[kz], W2, H2, Zc2);
#pragma unroll
                for (int q = 0; q < 5; ++q) sum[q] += sh[q * SH::SIZE];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) m[q * (size_t)N + cell] = sum[q];
}

// ------------------------------------------------------------ readout

// lap rho from the moment field (for the readout force).
template <int D, typename R>
__global__ void __launch_bounds__(256) k_lap_field(const R *__restrict__ m, R *__restrict__ lap, int nx, int ny, int nz)
{
    constexpr int HZ = Lat<D>::HZ;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const R c = m[(long)x + (long)nx * ((long)y + (long)ny * z)];
    R acc = R(0);
    for (int dz = -HZ; dz <= HZ; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const R w = w1<R>(dx) * w1<R>(dy) * (D == 3 ? w1<R>(dz) : R(1));
                const long n = (long)wrapi(x + dx, nx) + (long)nx * ((long)wrapi(y + dy, ny) + (long)ny * wrapi(z + dz, nz));
                acc += (R(6) * w) * (m[n] - c);
            }
    lap[(long)x + (long)nx * ((long)y + (long)ny * z)] = acc;
}

// Per-cell readout state: rho, u, RT, F, grad rho (all from the moment field
// and its Laplacian, radius 1).
template <int D, typename R>
struct CellState {
    R rho, u[3], RT, F[3], grad[3], rhoE;
};

template <int D, typename R>
__device__ inline CellState<D, R> cell_state(const R *__restrict__ m, const R *__restrict__ lap, long N, int x, int y,
                                             int z, int nx, int ny, int nz, R a, R kappa)
{
    constexpr int HZ = Lat<D>::HZ;
    CellState<D, R> s;
    const long cell = (long)x + (long)nx * ((long)y + (long)ny * z);
    s.rho = m[cell];
    R g2[3] = {R(0), R(0), R(0)}, gl[3] = {R(0), R(0), R(0)}, gr[3] = {R(0), R(0), R(0)};
    for (int dz = -HZ; dz <= HZ; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const R w = R(3) * w1<R>(dx) * w1<R>(dy) * (D == 3 ? w1<R>(dz) : R(1));
                const long n = (long)wrapi(x + dx, nx) + (long)nx * ((long)wrapi(y + dy, ny) + (long)ny * wrapi(z + dz, nz));
                const R r = m[n], l = lap[n];
                const int cc[3] = {dx, dy, dz};
                for (int ax = 0; ax < D; ++ax) {
                    g2[ax] += w * R(cc[ax]) * (r * r);
                    gl[ax] += w * R(cc[ax]) * l;
                    gr[ax] += w * R(cc[ax]) * r;
                }
            }
    R uF = R(0), u2 = R(0);
    for (int ax = 0; ax < 3; ++ax) {
        s.F[ax] = (ax < D) ? a * g2[ax] + kappa * s.rho * gl[ax] : R(0);
        s.grad[ax] = gr[ax];
        s.u[ax] = (ax < D) ? (m[(ax + 1) * N + cell] + R(0.5) * s.F[ax]) / s.rho : R(0);
        uF += s.u[ax] * s.F[ax];
        u2 += s.u[ax] * s.u[ax];
    }
    s.rhoE = m[(D + 1) * N + cell] + R(0.5) * uF;
    s.RT = (R(2) / R(3)) * (s.rhoE / s.rho - R(0.5) * u2);
    return s;
}

template <int D, typename R, typename O>
__global__ void __launch_bounds__(256) k_readout(const R *__restrict__ m, const R *__restrict__ lap, O *__restrict__ rho_out,
                                                 O *__restrict__ u_out, O *__restrict__ T_out, int nx, int ny, int nz,
                                                 R a, R kappa, R Rgas)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const long N = (long)nx * ny * nz;
    const long cell = (long)x + (long)nx * ((long)y + (long)ny * z);
    CellState<D, R> s = cell_state<D, R>(m, lap, N, x, y, z, nx, ny, nz, a, kappa);
    if (rho_out) rho_out[cell] = (O)s.rho;
    if (T_out) T_out[cell] = (O)(s.RT / Rgas);
    if (u_out)
        for (int aa = 0; aa < D; ++aa) u_out[aa * N + cell] = (O)s.u[aa];
}

// ------------------------------------------------------- FP64 reductions

// Block-level FP64 reduction of NV values in a fixed tree, one partial per
// block stored value-major: partial[k * gridDim.x + blockIdx.x].
// Op: 0 = sum, 1 = max, 2 = min.
__device__ inline double red_op(int op, double x, double y) { return op == 0 ? x + y : op == 1 ? fmax(x, y) : fmin(x, y); }

template <int NV>
__device__ inline void block_reduce_store(double v[NV], const int ops[NV], double *__restrict__ partial)
{
    __shared__ double s_red[NV][16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        for (int off = 32; off > 0; off >>= 1) x = red_op(ops[k], x, __shfl_xor(x, off, 64));
        if (lane == 0) s_red[k][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        double x = s_red[k][0];
        for (int w = 1; w < nw; ++w) x = red_op(ops[k], x, s_red[k][w]);
        partial[(long)k * gridDim.x + blockIdx.x] = x;
    }
}

// Final pass: block k reduces the nblocks partials of value k (coalesced,
// 256 threads, fixed order) into out[k].
static __global__ void __launch_bounds__(256) k_reduce_final(const double *__restrict__ partial, long nblocks, const int4 ops_lo,
                                                      const int4 ops_hi, double *__restrict__ out)
{
    __shared__ double s[256];
    const int k = blockIdx.x;
    const int ops[8] = {ops_lo.x, ops_lo.y, ops_lo.z, ops_lo.w, ops_hi.x, ops_hi.y, ops_hi.z, ops_hi.w};
    const int op = ops[k < 8 ? k : 0];
    double x = op == 0 ? 0.0 : op == 1 ? -1e300 : 1e300;
    for (long b = threadIdx.x; b < nblocks; b += 256) x = red_op(op, x, partial[(long)k * nblocks + b]);
    s[threadIdx.x] = x;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] = red_op(op, s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = s[0];
}

// Global sums of the readout state (FP64 accumulation), one cell per thread
// over a flat index.
template <int D, int S>
__global__ void __launch_bounds__(256) k_sums(const StoreT<S> *__restrict__ pop, const RealT<S> *__restrict__ m,
                                              const RealT<S> *__restrict__ lap, StepParams<RealT<S>> p,
                                              double *__restrict__ partial)
{
    using R = RealT<S>;
    constexpr int Q = Lat<D>::Q;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 1e300};
    const int ops[8] = {0, 0, 0, 0, 0, 0, 1, 2};
    if (cell < p.N) {
        const int x = (int)(cell % p.nx), y = (int)((cell / p.nx) % p.ny), z = (int)(cell / ((long)p.nx * p.ny));
        CellState<D, R> s = cell_state<D, R>(m, lap, p.N, x, y, z, p.nx, p.ny, p.nz, p.a, p.kappa);
        const double rho = s.rho;
        double u2 = 0.0, g2 = 0.0;
        v[0] = rho;
        for (int a = 0; a < D; ++a) {
            v[1 + a] = rho * (double)s.u[a];
            u2 += (double)s.u[a] * (double)s.u[a];
            g2 += (double)s.grad[a] * (double)s.grad[a];
        }
        v[4] = s.rhoE;
        v[5] = (double)s.rhoE - (double)p.a * rho * rho + 0.5 * (double)p.kappa * g2;
        v[6] = sqrt(u2);
        const int xs[3] = {x + 1 == p.nx ? 0 : x + 1, x, x == 0 ? p.nx - 1 : x - 1};
        const int ys[3] = {y + 1 == p.ny ? 0 : y + 1, y, y == 0 ? p.ny - 1 : y - 1};
        const int zs[3] = {z + 1 == p.nz ? 0 : z + 1, z, z == 0 ? p.nz - 1 : z - 1};
        // rho of the cell summed in FP64 over its decoded pulled populations:
        // the global sum is then the stored mass itself, free of the moment
        // field's per-cell rounding
        double fmin_ = 1e300, mass = 0.0;
        for (int i = 0; i < Q; ++i) {
            const long src = (long)xs[cx_of(i) + 1] + (long)p.nx * ((long)ys[cy_of(i) + 1] + (long)p.ny * zs[cz_d<D>(i) + 1]);
            const double f = Codec<S>::dec(pop[(long)i * p.ds + src], ref_at<D, S>(p, i, src));
            fmin_ = fmin(fmin_, f);
            mass += f;
        }
        v[0] = mass;
        v[7] = fmin_;
    }
    block_reduce_store<8>(v, ops, partial);
}

// Region means for coexistence / Laplace measurements.
// v = {sum rho_in, sum T_in, sum P_in, n_in, sum rho_out, sum T_out, sum P_out, n_out}
// plus a separate sum of rho over the whole lattice (sums[8]).
template <int D, typename R>
__global__ void __launch_bounds__(256) k_measure(const R *__restrict__ m, const R *__restrict__ lap, int nx, int ny, int nz,
                                                 int eos, R a, R b, R kappa, R Rgas, int kind, double g0, double g1, double g2,
                                                 double g3, double g4, double g5, double *__restrict__ partial)
{
    const long N = (long)nx * ny * nz;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int ops[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (cell < N) {
        const int x = (int)(cell % nx), y = (int)((cell / nx) % ny), z = (int)(cell / ((long)nx * ny));
        CellState<D, R> s = cell_state<D, R>(m, lap, N, x, y, z, nx, ny, nz, a, kappa);
        const double rho = s.rho, RT = s.RT;
        double Z = NAN;  // bulk pressure P = rho RT Z - a rho^2 (NaN outside the closure's range)
        enskog_z64(eos, (double)b, rho, &Z);
        const double P = rho * RT * Z - (double)a * rho * rho;
        int region = 0;  // 1 in, 2 out
        if (kind == EVLBM_MEASURE_SLAB) {
            if (x >= g0 && x < g1) region = 1;
            else if ((x >= g2 && x < g3) || (x >= g4 && x < g5)) region = 2;
        } else {
            const double dx = x - g0, dy = y - g1, dz = (D == 3) ? z - g2 : 0.0;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r < g3) region = 1;
            else if (r > g4) region = 2;
        }
        if (region == 1) {
            v[0] = rho; v[1] = RT / (double)Rgas; v[2] = P; v[3] = 1.0;
        } else if (region == 2) {
            v[4] = rho; v[5] = RT / (double)Rgas; v[6] = P; v[7] = 1.0;
        }
        v[8] = rho;
    }
    block_reduce_store<9>(v, ops, partial);
}

// Count cells whose density is not finite and positive.
template <typename R>
__global__ void __launch_bounds__(256) k_scan_nonfinite(const R *__restrict__ m, long N, int *__restrict__ flag)
{
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N) return;
    const R r = m[cell];
    if (!(r > R(0)) || !isfinite((double)r)) atomicAdd(flag, 1);
}

// Decode populations to FP64 / encode from FP64 (host I/O, checkpoints).
template <int D, int S>
__global__ void __launch_bounds__(256) k_decode(const StoreT<S> *__restrict__ pop, double *__restrict__ out, long N, int Q2,
                                                StepParams<RealT<S>> p)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * Q2) return;
    const int i = (int)(t / N);
    const long c = t - (long)i * N;
    out[t] = (double)Codec<S>::dec(pop[(long)i * p.ds + c], ref_at<D, S>(p, i, c));
}

template <int D, int S>
__global__ void __launch_bounds__(256) k_encode(const double *__restrict__ in, StoreT<S> *__restrict__ pop, long N, int Q2,
                                                StepParams<RealT<S>> p)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * Q2) return;
    const int i = (int)(t / N);
    const long c = t - (long)i * N;
    const float4 rs = ref_state_at<S>(p, c);
    pop[(long)i * p.ds + c] = Codec<S>::enc((RealT<S>)in[t], ref_enc<D, S>(i, rs, ref_inv_of<S, RealT<S>>(rs)));
}

// Validate initial fields: rho > 0 inside the range of the pressure closure
// (b rho < 1 for van der Waals, b rho < 4 for Carnahan-Starling), T > 0, finite.
static __global__ void __launch_bounds__(256) k_validate(const double *__restrict__ rho, const double *__restrict__ T, long N,
                                                  int eos, double b, int *__restrict__ flag)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const double r = rho[t], tt = T[t];
    double Z;
    if (!isfinite(r) || !isfinite(tt)) atomicOr(flag, 2);
    else if (!(r > 0.0) || !enskog_z64(eos, b, r, &Z) || !(tt > 0.0)) atomicOr(flag, 1);
}

// Z(rho) = P_E/(rho R T) in the arithmetic type V (enskog, enskog_z64).
template <typename V>
__device__ inline V enskog_Z(int eos, V b, V rho)
{
    if constexpr (sizeof(V) == 4) {
        return enskog<V>(eos, b, rho).Z;
    } else {
        V Z = V(NAN);
        enskog_z64(eos, b, rho, &Z);
        return Z;
    }
}

// 16-bit deviation storage: reference state of every cell (ref_state_of)
// from initial fields (rho, T), theta = RT Z(rho).
template <int D>
__global__ void __launch_bounds__(256) k_ref_from_fields(const double *__restrict__ rho, const double *__restrict__ T,
                                                         long N, double Rg, int eos, double b,
                                                         float4 *__restrict__ refst)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const double RT = Rg * T[t];
    refst[t] = ref_state_of<D>(rho[t], RT * enskog_Z<double>(eos, b, rho[t]), 1.5 * RT);
}

// The same from populations f, g at rest in the cell's own frame: rho = sum f,
// j = sum c f, K = sum g/rho - |j|^2/(2 rho^2) = (3/2) RT, in the arithmetic
// type V (the reference only sets the scale of the stored deviations).
template <int D, typename V>
__device__ inline float4 ref_state(const V *f, const V *g, int eos, V b)
{
    constexpr int Q = Lat<D>::Q;
    V rho = V(0), e = V(0), j[3] = {V(0), V(0), V(0)};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        e += g[i];
        j[0] += V(cx_of(i)) * f[i];
        j[1] += V(cy_of(i)) * f[i];
        j[2] += V(cz_d<D>(i)) * f[i];
    }
    const V K = e / rho - V(0.5) * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / (rho * rho);
    return ref_state_of<D, V>(rho, (V(2) / V(3)) * K * enskog_Z<V>(eos, b, rho), K);
}

// From decoded populations in the dense host layout ([Q][N] f, then g).
template <int D>
__global__ void __launch_bounds__(256) k_ref_from_pops(const double *__restrict__ pops, long N, int eos, double b,
                                                       float4 *__restrict__ refst)
{
    constexpr int Q = Lat<D>::Q;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    double f[Q], g[Q];
    for (int i = 0; i < Q; ++i) {
        f[i] = pops[(long)i * N + t];
        g[i] = pops[(long)(Q + i) * N + t];
    }
    refst[t] = ref_state<D>(f, g, eos, b);
}

// Re-reference in place: decode the 2Q values stored at a cell with its old
// reference, take the state they carry as the new reference, encode again.
// Each thread owns one cell (values stored at a cell are encoded with that
// cell's reference).  p.refst is the old state; refst receives the new one
// (the same array).
template <int D, int S>
__global__ void __launch_bounds__(256) k_rereference(StoreT<S> *__restrict__ pop, float4 *refst,
                                                     StepParams<RealT<S>> p)
{
    constexpr int Q = Lat<D>::Q;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.N) return;
    using R = RealT<S>;
    R f[Q], g[Q];
    for (int i = 0; i < Q; ++i) {
        f[i] = Codec<S>::dec(pop[(long)i * p.ds + t], ref_at<D, S>(p, i, t));
        g[i] = Codec<S>::dec(pop[(long)(Q + i) * p.ds + t], ref_at<D, S>(p, Q + i, t));
    }
    const float4 rs = ref_state<D, R>(f, g, p.eos, p.b);
    refst[t] = rs;
    const RefInv<RealT<S>> inv = ref_inv_of<S, RealT<S>>(rs);
    // re-encode keeping the cell's mass and energy: rest + opposite pair close
    // the balances as in the collision
    constexpr int REST = (Q - 1) / 2, SA = Q - 1, SB = 0;
    const PtrPops<StoreT<S>> pops{pop, pop, p.ds};
    const unsigned cb = (unsigned)t * (unsigned)sizeof(StoreT<S>);
    Compensated<R> mf{f[REST], R(0)}, mg{g[REST], R(0)};  // Fast2Sum from the largest population
    for (int i = 0; i < Q; ++i) {
        if (i == REST) continue;
        mf.add(f[i]);
        mg.add(g[i]);
        if (i == SA || i == SB) continue;
        const Ref<R> rf = ref_enc<D, S>(i, rs, inv), rg = ref_enc<D, S>(Q + i, rs, inv);
        const StoreT<S> fq = Codec<S>::enc(f[i], rf), gq = Codec<S>::enc(g[i], rg);
        pops.st(i, cb, fq);
        pops.st(Q + i, cb, gq);
        mf.add(-Codec<S>::dec(fq, rf));
        mg.add(-Codec<S>::dec(gq, rg));
    }
    R cd[3];
    close_three<S>(pops, cb, REST, SA, SB, mf, f[SA], f[SB], ref_enc<D, S>(REST, rs, inv),
                   ref_enc<D, S>(SA, rs, inv), ref_enc<D, S>(SB, rs, inv), cd);
    close_three<S>(pops, cb, Q + REST, Q + SA, Q + SB, mg, g[SA], g[SB], ref_enc<D, S>(Q + REST, rs, inv),
                   ref_enc<D, S>(Q + SA, rs, inv), ref_enc<D, S>(Q + SB, rs, inv), cd);
}

static __global__ void __launch_bounds__(256) k_f64_to_f32(const double *__restrict__ in, float *__restrict__ out, long n)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = (float)in[t];
}

static __global__ void __launch_bounds__(256) k_f32_to_f64(const float *__restrict__ in, double *__restrict__ out, long n)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = (double)in[t];
}

}  // namespace evlbm
