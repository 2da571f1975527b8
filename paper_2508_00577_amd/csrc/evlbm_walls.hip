// Diffuse walls normal to x for the thermal Couette flow of the paper's
// second validation (the paragraph after eq. P0E, Fig. 2): a wall half a
// cell outside the first cell (x = -1/2, at rest) and one half a cell
// outside the last (x = nx - 1/2, moving with U_w along y), both at T_w;
// periodic in y and z.  The paper gives the wall values only; the scheme
// taken here:
//   - streaming: a population entering a cell from a wall is the wall's
//     equilibrium (eq. feq, eq. geq at u_w, RT_w and theta_w = RT_w Z(rho) at
//     the cell's stored density) times the density that makes the mass it
//     carries equal the mass of the cell's populations heading into the wall
//     in the same step (diffuse reflection: mass conserving, fully
//     accommodating);
//   - stencils: a field beyond a wall is the linear extrapolation through the
//     two cells next to it, phi(e) + k (phi(e) - phi(e -+ 1)) at distance k.
// A wall step is four launches: the pull with the re-emission (moments and
// the streamed populations), the Laplacian of rho, the force and half-step
// fields, and the corrections with the collision of eq. pre_LBM
// (collide_pulled, shared with the periodic steps).  FP64 and FP32 storage.
#include <cmath>
#include <utility>

#include "evlbm_internal.hpp"
#include "evlbm_params.hpp"
#include "lbm_kernels.hpp"

namespace evlbm {

template <typename R>
StepParams<R> make_params(const evlbm_lattice *h);

// Value of field f ([N], x fastest) at (x + dx, y + dy, z + dz): periodic in
// y and z; beyond a wall in x the linear extrapolation through the two cells
// next to it.
template <typename R>
__device__ inline R wall_field(const R *__restrict__ f, int x, int y, int z, int dx, int dy, int dz, int nx, int ny,
                               int nz)
{
    const long yz = (long)nx * ((long)wrapi(y + dy, ny) + (long)ny * wrapi(z + dz, nz));
    const int xx = x + dx;
    if (xx < 0) {
        const R e = f[yz], in = f[yz + 1];
        return e + R(-xx) * (e - in);
    }
    if (xx >= nx) {
        const R e = f[yz + nx - 1], in = f[yz + nx - 2];
        return e + R(xx - (nx - 1)) * (e - in);
    }
    return f[yz + xx];
}

// Isotropic derivative d_a phi = 3 sum_i w_i c_ia phi(x + c_i) and Laplacian
// 6 sum_i w_i (phi(x + c_i) - phi(x)) with the wall ghosts (SQ: of phi^2).
template <int D, int A, bool SQ, typename R>
__device__ inline R wall_grad(const R *__restrict__ f, int x, int y, int z, int nx, int ny, int nz)
{
    constexpr int HZ = Lat<D>::HZ;
    R acc = R(0);
    for (int dz = -HZ; dz <= HZ; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int ca = (A == 0) ? dx : (A == 1) ? dy : dz;
                if (ca == 0) continue;
                const R w = R(3) * w1<R>(dx) * w1<R>(dy) * (D == 3 ? w1<R>(dz) : R(1));
                R v;
                if constexpr (SQ) {
                    // the field is rho^2: its ghost is the extrapolation of rho^2
                    const long yz = (long)nx * ((long)wrapi(y + dy, ny) + (long)ny * wrapi(z + dz, nz));
                    const int xx = x + dx;
                    if (xx < 0 || xx >= nx) {
                        const long e = yz + (xx < 0 ? 0 : nx - 1), in = yz + (xx < 0 ? 1 : nx - 2);
                        const R se = f[e] * f[e], si = f[in] * f[in];
                        v = se + R(xx < 0 ? -xx : xx - (nx - 1)) * (se - si);
                    } else {
                        v = f[yz + xx] * f[yz + xx];
                    }
                } else {
                    v = wall_field(f, x, y, z, dx, dy, dz, nx, ny, nz);
                }
                acc += (w * R(ca)) * v;
            }
    return acc;
}

template <int D, typename R>
__device__ inline R wall_lap(const R *__restrict__ f, int x, int y, int z, int nx, int ny, int nz)
{
    constexpr int HZ = Lat<D>::HZ;
    const R centre = f[(long)x + (long)nx * ((long)y + (long)ny * z)];
    R acc = R(0);
    for (int dz = -HZ; dz <= HZ; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const R w = R(6) * w1<R>(dx) * w1<R>(dy) * (D == 3 ? w1<R>(dz) : R(1));
                acc += w * (wall_field(f, x, y, z, dx, dy, dz, nx, ny, nz) - centre);
            }
    return acc;
}

// Pull with the walls: fh[2Q][N] (f then g, decoded) and the moments rho, j,
// e into m ([D+2][N]).
template <int D, int S>
__global__ void __launch_bounds__(256) k_wall_pull(const StoreT<S> *__restrict__ pop, RealT<S> *__restrict__ fh,
                                                   RealT<S> *__restrict__ m, StepParams<RealT<S>> p, double RTw,
                                                   double Uw)
{
    using R = RealT<S>;
    constexpr int Q = Lat<D>::Q;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= p.N) return;
    const int x = (int)(cell % p.nx), y = (int)((cell / p.nx) % p.ny), z = (int)(cell / ((long)p.nx * p.ny));
    // wall re-emission of a cell next to a wall (side -1: x = -1/2, +1: x = nx - 1/2)
    R rho_w[2] = {R(0), R(0)}, fe[2][3][3], xe[2][3][3], hRT = R(0);
    for (int s = 0; s < 2; ++s) {
        const int side = s ? 1 : -1;
        if ((side < 0 && x != 0) || (side > 0 && x != p.nx - 1)) continue;
        R rho = R(0), out = R(0);
        for (int i = 0; i < Q; ++i) {
            const R f = Codec<S>::dec(pop[(long)i * p.ds + cell], Ref<R>{R(0), R(1), R(1)});
            rho += f;
            if (cx_of(i) == side) out += f;
        }
        const R RT = (R)RTw, theta = RT * enskog_Z<R>(p.eos, p.b, rho);
        const R uw[3] = {R(0), side > 0 ? (R)Uw : R(0), R(0)};
        for (int a = 0; a < 3; ++a) {
            if (a < D) {
                psi3<R>(uw[a], theta + uw[a] * uw[a], fe[s][a]);
                chi3<R>(uw[a], theta, xe[s][a]);
            } else {
                fe[s][a][0] = fe[s][a][2] = R(0);
                fe[s][a][1] = R(1);
                xe[s][a][0] = xe[s][a][1] = xe[s][a][2] = R(0);
            }
        }
        R in = R(0);
        for (int i = 0; i < Q; ++i)
            if (cx_of(i) == -side) in += fe[s][0][cx_of(i) + 1] * fe[s][1][cy_of(i) + 1] * fe[s][2][cz_d<D>(i) + 1];
        rho_w[s] = out / in;
        hRT = R(1.5) * RT;
    }
    R mo[5] = {R(0), R(0), R(0), R(0), R(0)};
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_of(i), cy = cy_of(i), cz = cz_d<D>(i);
        const int sx = x - cx;
        R f, g;
        if (sx < 0 || sx >= p.nx) {
            const int s = sx < 0 ? 0 : 1;
            const int kx = cx + 1, ky = cy + 1, kz = cz + 1;
            const R pe = fe[s][0][kx] * fe[s][1][ky] * fe[s][2][kz];
            f = rho_w[s] * pe;
            g = rho_w[s] * ((hRT * fe[s][0][kx] + xe[s][0][kx]) * fe[s][1][ky] * fe[s][2][kz] +
                            fe[s][0][kx] * (xe[s][1][ky] * fe[s][2][kz] + fe[s][1][ky] * xe[s][2][kz]));
        } else {
            const long src = (long)sx + (long)p.nx * ((long)wrapi(y - cy, p.ny) + (long)p.ny * wrapi(z - cz, p.nz));
            f = Codec<S>::dec(pop[(long)i * p.ds + src], Ref<R>{R(0), R(1), R(1)});
            g = Codec<S>::dec(pop[(long)(Q + i) * p.ds + src], Ref<R>{R(0), R(1), R(1)});
        }
        fh[(long)i * p.N + cell] = f;
        fh[(long)(Q + i) * p.N + cell] = g;
        mo[0] += f;
        mo[1] += R(cx) * f;
        mo[2] += R(cy) * f;
        mo[3] += R(cz) * f;
        mo[4] += g;
    }
    m[cell] = mo[0];
    for (int a = 0; a < D; ++a) m[(1 + a) * p.N + cell] = mo[1 + a];
    m[(D + 1) * p.N + cell] = mo[4];
}

template <int D, typename R>
__global__ void __launch_bounds__(256) k_wall_lap(const R *__restrict__ m, R *__restrict__ lap, int nx, int ny, int nz)
{
    const long N = (long)nx * ny * nz;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N) return;
    const int x = (int)(cell % nx), y = (int)((cell / nx) % ny), z = (int)(cell / ((long)nx * ny));
    lap[cell] = wall_lap<D, R>(m, x, y, z, nx, ny, nz);
}

// Force (eq. EVforce1 under eq. P0E) and half-step fields (eq. u_shift,
// eq. T_shift) with the wall ghosts: fld = {u (D), M = rho u (u^2 + 3 theta
// - 1) (D), F (D), theta - RT, K = (3/2) RT}, [3D + 2][N].
template <int D, typename R>
__global__ void __launch_bounds__(256) k_wall_fields(const R *__restrict__ m, const R *__restrict__ lap,
                                                     R *__restrict__ fld, StepParams<R> p)
{
    const long N = p.N;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N) return;
    const int x = (int)(cell % p.nx), y = (int)((cell / p.nx) % p.ny), z = (int)(cell / ((long)p.nx * p.ny));
    const R rho = m[cell];
    R F[3] = {R(0), R(0), R(0)};
    F[0] = p.a * wall_grad<D, 0, true, R>(m, x, y, z, p.nx, p.ny, p.nz) +
           p.kappa * rho * wall_grad<D, 0, false, R>(lap, x, y, z, p.nx, p.ny, p.nz);
    F[1] = p.a * wall_grad<D, 1, true, R>(m, x, y, z, p.nx, p.ny, p.nz) +
           p.kappa * rho * wall_grad<D, 1, false, R>(lap, x, y, z, p.nx, p.ny, p.nz);
    if (D == 3)
        F[2] = p.a * wall_grad<D, 2, true, R>(m, x, y, z, p.nx, p.ny, p.nz) +
               p.kappa * rho * wall_grad<D, 2, false, R>(lap, x, y, z, p.nx, p.ny, p.nz);
    const R ir = R(1) / rho;
    R u[3] = {R(0), R(0), R(0)}, uF = R(0), u2 = R(0);
    for (int a = 0; a < D; ++a) {
        u[a] = (m[(1 + a) * N + cell] + R(0.5) * F[a]) * ir;
        uF += u[a] * F[a];
        u2 += u[a] * u[a];
    }
    const R K = (m[(D + 1) * N + cell] + R(0.5) * uF) * ir - R(0.5) * u2;
    const R RT = K * (R(2) / R(3));
    const R theta = RT * enskog_Z<R>(p.eos, p.b, rho);
    for (int a = 0; a < D; ++a) {
        fld[(long)a * N + cell] = u[a];
        fld[(long)(D + a) * N + cell] = rho * u[a] * (u[a] * u[a] + R(3) * theta - R(1));
        fld[(long)(2 * D + a) * N + cell] = F[a];
    }
    fld[(long)(3 * D) * N + cell] = theta - RT;
    fld[(long)(3 * D + 1) * N + cell] = K;
}

// Corrections (eq. correction_u, correction_gamma, correction_q) with the
// wall ghosts, then the shifted state, equilibria and update of eq. pre_LBM
// (collide_pulled) from the streamed populations fh into dst.
template <int D, int S, bool VPR>
__global__ void __launch_bounds__(256) k_wall_collide(const RealT<S> *__restrict__ fh, const RealT<S> *__restrict__ m,
                                                      const RealT<S> *__restrict__ fld, StoreT<S> *__restrict__ dst,
                                                      StepParams<RealT<S>> p)
{
    using R = RealT<S>;
    using T = StoreT<S>;
    static_assert(sizeof(T) == sizeof(R), "walls take FP64 or FP32 storage");
    constexpr int Q = Lat<D>::Q;
    const long N = p.N;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N) return;
    const int x = (int)(cell % p.nx), y = (int)((cell / p.nx) % p.ny), z = (int)(cell / ((long)p.nx * p.ny));
    const R rho = m[cell], inv_rho = rcp(rho);
    const R K = fld[(long)(3 * D + 1) * N + cell];
    const R RT = K * (R(2) / R(3));
    const Enskog<R> ez = enskog(p.eos, p.b, rho);
    const R theta = RT * ez.Z, P0 = rho * theta;
    R u[3] = {R(0), R(0), R(0)}, F[3] = {R(0), R(0), R(0)}, Phi[3] = {R(0), R(0), R(0)}, qp[3] = {R(0), R(0), R(0)};
    for (int a = 0; a < D; ++a) {
        u[a] = fld[(long)a * N + cell];
        F[a] = fld[(long)(2 * D + a) * N + cell];
    }
    const R *fu = fld, *fM = fld + (long)D * N, *ftd = fld + (long)(3 * D) * N;
    R divu = wall_grad<D, 0, false, R>(fu, x, y, z, p.nx, p.ny, p.nz) +
             wall_grad<D, 1, false, R>(fu + N, x, y, z, p.nx, p.ny, p.nz);
    if (D == 3) divu += wall_grad<D, 2, false, R>(fu + 2 * N, x, y, z, p.nx, p.ny, p.nz);
    const R Phip = P0 * ez.g5 * divu;
    Phi[0] = p.sphi * wall_grad<D, 0, false, R>(fM, x, y, z, p.nx, p.ny, p.nz) + Phip;
    Phi[1] = p.sphi * wall_grad<D, 1, false, R>(fM + N, x, y, z, p.nx, p.ny, p.nz) + Phip;
    qp[0] = p.lambda * (P0 * wall_grad<D, 0, false, R>(ftd, x, y, z, p.nx, p.ny, p.nz) + u[0] * Phip);
    qp[1] = p.lambda * (P0 * wall_grad<D, 1, false, R>(ftd, x, y, z, p.nx, p.ny, p.nz) + u[1] * Phip);
    if (D == 3) {
        Phi[2] = p.sphi * wall_grad<D, 2, false, R>(fM + 2 * N, x, y, z, p.nx, p.ny, p.nz) + Phip;
        qp[2] = p.lambda * (P0 * wall_grad<D, 2, false, R>(ftd, x, y, z, p.nx, p.ny, p.nz) + u[2] * Phip);
    }
    T fr[Q], gr[Q];
    for (int i = 0; i < Q; ++i) {
        fr[i] = (T)fh[(long)i * N + cell];
        gr[i] = (T)fh[(long)(Q + i) * N + cell];
    }
    // every "pull source" of the accessor is the cell itself: the values are
    // already streamed; the stores go to the cell's byte offset in dst
    PullOffsets o;
    const unsigned cb = (unsigned)cell * (unsigned)sizeof(T);
    for (int k = 0; k < 3; ++k) {
        o.ox[k] = cb;
        o.oy[k] = 0u;
        o.oz[k] = 0u;
    }
    const PtrPops<T> pops{dst, dst, p.ds};
    collide_pulled<D, S, PtrPops<T>, NoSink, VPR>(fr, gr, pops, p, o, rho, inv_rho, K, ez.Z, theta, u, F, Phi, qp);
}

template <int D, typename R, typename O>
__global__ void __launch_bounds__(256) k_wall_readout(const R *__restrict__ m, const R *__restrict__ fld, long N, int Dd,
                                                      R Rgas, O *__restrict__ rho, O *__restrict__ u, O *__restrict__ T)
{
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= N) return;
    if (rho) rho[cell] = (O)m[cell];
    if (T) T[cell] = (O)(fld[(long)(3 * D + 1) * N + cell] * (R(2) / R(3)) / Rgas);
    if (u)
        for (int a = 0; a < D; ++a) u[(long)a * N + cell] = (O)fld[(long)a * N + cell];
}

// FP64 sums of the wall state: sum rho (the streamed populations: the stored
// mass), sum rho u, sum rho E, sum [rho E - a rho^2 + (kappa/2)|grad rho|^2]
// (wall ghosts), max |u|, min of the streamed f.
template <int D, typename R>
__global__ void __launch_bounds__(256) k_wall_sums(const R *__restrict__ fh, const R *__restrict__ m,
                                                   const R *__restrict__ fld, StepParams<R> p, double *__restrict__ partial)
{
    constexpr int Q = Lat<D>::Q;
    const long N = p.N;
    const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int ops[8] = {0, 0, 0, 0, 0, 0, 1, 2};
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 1e300};
    if (cell < N) {
        const int x = (int)(cell % p.nx), y = (int)((cell / p.nx) % p.ny), z = (int)(cell / ((long)p.nx * p.ny));
        double mass = 0.0, fmin_ = 1e300, u2 = 0.0, g2 = 0.0;
        for (int i = 0; i < Q; ++i) {
            const double f = fh[(long)i * N + cell];
            mass += f;
            fmin_ = fmin(fmin_, f);
        }
        const double rho = m[cell];
        for (int a = 0; a < D; ++a) {
            const double ua = fld[(long)a * N + cell];
            v[1 + a] = rho * ua;
            u2 += ua * ua;
        }
        const double gx = wall_grad<D, 0, false, R>(m, x, y, z, p.nx, p.ny, p.nz);
        const double gy = wall_grad<D, 1, false, R>(m, x, y, z, p.nx, p.ny, p.nz);
        const double gz = D == 3 ? (double)wall_grad<D, 2, false, R>(m, x, y, z, p.nx, p.ny, p.nz) : 0.0;
        g2 = gx * gx + gy * gy + gz * gz;
        const double rhoE = rho * ((double)fld[(long)(3 * D + 1) * N + cell] + 0.5 * u2);
        v[0] = mass;
        v[4] = rhoE;
        v[5] = rhoE - (double)p.a * rho * rho + 0.5 * (double)p.kappa * g2;
        v[6] = sqrt(u2);
        v[7] = fmin_;
    }
    block_reduce_store<8>(v, ops, partial);
}

template <int D, int S>
struct WallOps {
    using T = StoreT<S>;
    using R = RealT<S>;
    static unsigned blocks(const evlbm_lattice *h) { return (unsigned)((h->N + 255) / 256); }
    // pull, Laplacian and fields of the current state: m, lap, wall_fld, wall_fh
    static void analyse(evlbm_lattice *h)
    {
        const StepParams<R> p = make_params<R>(h);
        hipLaunchKernelGGL((k_wall_pull<D, S>), dim3(blocks(h)), dim3(256), 0, h->stream, (const T *)h->buf[h->cur],
                           (R *)h->wall_fh, (R *)h->m, p, h->R * h->Tw, h->Uw);
        hipLaunchKernelGGL((k_wall_lap<D, R>), dim3(blocks(h)), dim3(256), 0, h->stream, (const R *)h->m, (R *)h->lap,
                           h->nx, h->ny, h->nz);
        hipLaunchKernelGGL((k_wall_fields<D, R>), dim3(blocks(h)), dim3(256), 0, h->stream, (const R *)h->m,
                           (const R *)h->lap, (R *)h->wall_fld, p);
    }
    static void step(evlbm_lattice *h)
    {
        analyse(h);
        if (h->prandtl != 1.0)
            hipLaunchKernelGGL((k_wall_collide<D, S, true>), dim3(blocks(h)), dim3(256), 0, h->stream,
                               (const R *)h->wall_fh, (const R *)h->m, (const R *)h->wall_fld, (T *)h->buf[1 - h->cur],
                               make_params<R>(h));
        else
            hipLaunchKernelGGL((k_wall_collide<D, S, false>), dim3(blocks(h)), dim3(256), 0, h->stream,
                               (const R *)h->wall_fh, (const R *)h->m, (const R *)h->wall_fld, (T *)h->buf[1 - h->cur],
                               make_params<R>(h));
    }
    template <typename O>
    static void readout(evlbm_lattice *h, O *rho, O *u, O *T0)
    {
        analyse(h);
        hipLaunchKernelGGL((k_wall_readout<D, R, O>), dim3(blocks(h)), dim3(256), 0, h->stream, (const R *)h->m,
                           (const R *)h->wall_fld, h->N, D, (R)h->R, rho, u, T0);
    }
    static void sums(evlbm_lattice *h, double *partial)
    {
        analyse(h);
        hipLaunchKernelGGL((k_wall_sums<D, R>), dim3(blocks(h)), dim3(256), 0, h->stream, (const R *)h->wall_fh,
                           (const R *)h->m, (const R *)h->wall_fld, make_params<R>(h), partial);
    }
};

template <class F>
static void wall_dispatch(evlbm_lattice *h, F &&f)
{
    if (h->D == 2 && h->storage == EVLBM_F64) f(WallOps<2, EVLBM_F64>());
    else if (h->D == 2 && h->storage == EVLBM_F32) f(WallOps<2, EVLBM_F32>());
    else if (h->D == 3 && h->storage == EVLBM_F64) f(WallOps<3, EVLBM_F64>());
    else if (h->D == 3 && h->storage == EVLBM_F32) f(WallOps<3, EVLBM_F32>());
}

void wall_step(evlbm_lattice *h)
{
    wall_dispatch(h, [&](auto ops) { decltype(ops)::step(h); });
}

void wall_analyse(evlbm_lattice *h)
{
    wall_dispatch(h, [&](auto ops) { decltype(ops)::analyse(h); });
}

int wall_read_moments(evlbm_lattice *h, void *rho, void *u, void *T, int where, double *scratch3)
{
    if (where == EVLBM_DEVICE_F32) {
        wall_dispatch(h, [&](auto ops) { decltype(ops)::template readout<float>(h, (float *)rho, (float *)u, (float *)T); });
    } else {
        double *r = (double *)rho, *uu = (double *)u, *t = (double *)T;
        if (where == EVLBM_HOST_F64) {
            r = scratch3;
            t = scratch3 + h->N;
            uu = scratch3 + 2 * h->N;
        }
        wall_dispatch(h, [&](auto ops) { decltype(ops)::template readout<double>(h, r, uu, t); });
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "wall readout");
    return EVLBM_OK;
}

void wall_sums(evlbm_lattice *h, double *partial)
{
    wall_dispatch(h, [&](auto ops) { decltype(ops)::sums(h, partial); });
}

}  // namespace evlbm

extern "C" int evlbm_set_walls(evlbm_t h, int enable, double T_wall, double U_wall)
{
    using namespace evlbm;
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    auto drop_graphs = [h] {
        for (int k = 0; k < 2; ++k) {
            if (h->graph_exec_par[k]) (void)hipGraphExecDestroy(h->graph_exec_par[k]);
            h->graph_exec_par[k] = nullptr;
        }
    };
    if (!enable) {
        h->walls = false;
        h->m_valid = false;
        drop_graphs();  // the captured steps launch the wall kernels
        return EVLBM_OK;
    }
    if (h->storage != EVLBM_F64 && h->storage != EVLBM_F32)
        return fail(EVLBM_EINVAL, "walls take FP64 or FP32 storage");
    if (h->nx < 2 || !(T_wall > 0) || !std::isfinite(U_wall))
        return fail(EVLBM_EINVAL, "walls need nx >= 2, T_wall > 0 and a finite wall speed");
    const size_t rb = real_bytes(h->storage);
    if (!h->wall_fh || !h->wall_fld) {
        hipError_t e = h->wall_fh ? hipSuccess : hipMalloc(&h->wall_fh, rb * 2 * h->Q * h->N);
        if (e == hipSuccess) e = hipMalloc(&h->wall_fld, rb * (3 * h->D + 2) * h->N);
        if (e != hipSuccess) {
            (void)hipFree(h->wall_fh);
            h->wall_fh = nullptr;
            h->wall_fld = nullptr;
            return fail(EVLBM_ENOMEM, "wall work buffers: %s", hipGetErrorString(e));
        }
    }
    h->walls = true;
    h->Tw = T_wall;
    h->Uw = U_wall;
    h->m_valid = false;
    drop_graphs();
    return EVLBM_OK;
}
