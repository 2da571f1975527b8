// Initialisers of a lattice from the seeded synthetic states of the
// workloads (declared in include/evlbm.h): a flat liquid slab, a droplet with
// the tanh or the warm-start network's profile, and the network's droplet
// carrying a given total mass and total energy.  Every state starts at rest
// at a uniform temperature and goes through evlbm_init_fields (f = f^eq,
// g = g^eq of eq. feq and eq. geq).
#include <cmath>

#include "evlbm_internal.hpp"
#include "lbm_device.hpp"

namespace evlbm {

// splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): output k of the stream `seed` is the state
// seed + k * 0x9E3779B97F4A7C15 passed through the mixer
//   z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
//   z *= 0x94D049BB133111EB; z ^= z >> 31.
// Counter-based: cell c (linear index x + nx (y + ny z)) takes output c + 1,
// as a double on [0, 1) from its top 53 bits.
__host__ __device__ inline double splitmix_u01(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

// Multiplicative density noise: rho <- rho (1 + A U[-1, 1)).
__device__ inline double noisy(double rho, uint64_t seed, double A, long c)
{
    return A == 0.0 ? rho : rho * (1.0 + A * (2.0 * splitmix_u01(seed, (uint64_t)c) - 1.0));
}

// Flat slab along x between x0 and x1:
// rho = rho_v + (rho_l - rho_v)/2 [tanh((x - x0)/W) - tanh((x - x1)/W)].
__global__ void __launch_bounds__(256) k_slab(int nx, long n, double x0, double x1, double W, double rl, double rv,
                                              double T0, uint64_t seed, double A, double *__restrict__ rho,
                                              double *__restrict__ T)
{
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double x = (double)(c % nx);
    rho[c] = noisy(rv + 0.5 * (rl - rv) * (tanh((x - x0) / W) - tanh((x - x1) / W)), seed, A, c);
    T[c] = T0;
}

// Droplet of radius R centred at (cx, cy, cz) (2D distance when nz = 1):
// rho = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh((r - R)/W); with rho = null
// only T is written (the network supplies the profile).
__global__ void __launch_bounds__(256) k_tanh_droplet(int nx, int ny, int nz, double cx, double cy, double cz,
                                                      double R, double W, double rl, double rv, double T0,
                                                      uint64_t seed, double A, double *__restrict__ rho,
                                                      double *__restrict__ T, long n)
{
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long)nx * ny));
    const double dx = x - cx, dy = y - cy, dz = nz > 1 ? z - cz : 0.0;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (rho) rho[c] = noisy(0.5 * (rl + rv) - 0.5 * (rl - rv) * tanh((r - R) / W), seed, A, c);
    T[c] = T0;
}

// rho <- s * noisy(rho) (network profile: noise, then the mass scale), T <- T0.
__global__ void __launch_bounds__(256) k_noise_scale(double *__restrict__ rho, double *__restrict__ T, long n,
                                                     uint64_t seed, double A, double s, double T0)
{
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    rho[c] = s * noisy(rho[c], seed, A, c);
    T[c] = T0;
}

namespace {

// Critical point and coexistence densities of the handle's closure at T/Tc.
int coexistence_at(evlbm_t h, double Tr, double cp[3], double co[3])
{
    if (!(h->a > 0) || !(h->b > 0)) return fail(EVLBM_EINVAL, "initialisers need a two-phase fluid: a > 0 and b > 0");
    int rc = evlbm_eos_critical(h->eos, h->R, h->a, h->b, cp);
    if (rc) return rc;
    return evlbm_eos_coexistence(h->eos, h->R, h->a, h->b, Tr * cp[1], co);
}

// Device FP64 fields of a droplet: the network's profile when it passes the
// fallback checks, else the tanh profile; returns through used_mlp which.
int droplet_fields(evlbm_t h, double cx, double cy, double cz, double R, double Tr, int profile, evlbm_mlp_t mlp,
                   double width, uint64_t seed, double noise, double *drho, double *dT, bool *used)
{
    if (!(R > 0) || !(Tr > 0) || !(width > 0) || !(noise >= 0 && noise < 1))
        return fail(EVLBM_EINVAL, "bad droplet arguments (R, T/Tc, width > 0, 0 <= noise < 1)");
    if (profile != EVLBM_PROFILE_TANH && profile != EVLBM_PROFILE_MLP) return fail(EVLBM_EINVAL, "unknown profile");
    if (profile == EVLBM_PROFILE_MLP && !mlp) return fail(EVLBM_EINVAL, "MLP profile needs a network");
    double cp[3], co[3];
    int rc = coexistence_at(h, Tr, cp, co);
    if (rc) return rc;
    const double Tc = cp[1], rho_c = cp[0], rl = co[0], rv = co[1];
    bool mlp_ok = false;
    double hull[4];
    // the network takes (and its box holds) FP32 inputs: compare in FP32, so
    // that T/Tc = 0.95 lies inside a box trained up to 0.95f
    const double trf = (float)Tr, rf = (float)R;
    if (profile == EVLBM_PROFILE_MLP && evlbm_mlp_get_hull(mlp, hull) == EVLBM_OK && trf >= hull[0] &&
        trf <= hull[1] && rf >= hull[2] && rf <= hull[3]) {
        // radial probe r/R in [0, MLP_RMAX] (the field takes the value at
        // MLP_RMAX beyond it): finite, non-increasing (to 1e-3 rho_c) and
        // within [0.5 rho_v, 1.2 rho_l]
        const int np = 256;
        std::vector<float> X(3 * np), Y(np);
        for (int k = 0; k < np; ++k) {
            X[3 * k] = (float)Tr;
            X[3 * k + 1] = (float)R;
            X[3 * k + 2] = MLP_RMAX * k / (np - 1);
        }
        rc = evlbm_mlp_forward(mlp, X.data(), Y.data(), np);
        if (rc) return rc;
        mlp_ok = true;
        for (int k = 0; k < np; ++k) {
            const double v = rho_c * Y[k];
            if (!std::isfinite(v) || v < 0.5 * rv || v > 1.2 * rl) mlp_ok = false;
            if (k > 0 && rho_c * (Y[k] - Y[k - 1]) > 1e-3 * rho_c) mlp_ok = false;
        }
    }
    const long N = h->N;
    const unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_tanh_droplet, dim3(nb), dim3(256), 0, h->stream, h->nx, h->ny, h->nz, cx, cy, cz, R, width,
                       rl, rv, Tr * Tc, seed, noise, mlp_ok ? (double *)nullptr : drho, dT, N);
    hipError_t e = hipSuccess;
    if (mlp_ok) {
        // the network runs on its own stream: order it after the lattice stream and back
        e = hipStreamSynchronize(h->stream);
        if (e == hipSuccess) rc = evlbm_mlp_density_field(mlp, h->nx, h->ny, h->nz, cx, cy, cz, R, Tr, rho_c, drho);
        if (e == hipSuccess && rc == EVLBM_OK) e = hipStreamSynchronize(mlp_stream(mlp));
        if (e == hipSuccess && rc == EVLBM_OK)
            hipLaunchKernelGGL(k_noise_scale, dim3(nb), dim3(256), 0, h->stream, drho, dT, N, seed, noise, 1.0,
                               Tr * Tc);
    }
    if (e != hipSuccess) return hip_fail(e, "droplet fields");
    if (rc) return rc;
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "droplet fields");
    *used = mlp_ok;
    return EVLBM_OK;
}

// Device scratch for two FP64 fields, released by the caller with hipFree.
int two_fields(evlbm_t h, double **d)
{
    hipError_t e = hipMalloc(d, sizeof(double) * 2 * h->N);
    if (e != hipSuccess) return fail(EVLBM_ENOMEM, "initial fields: %s", hipGetErrorString(e));
    return EVLBM_OK;
}

}  // namespace
}  // namespace evlbm

using namespace evlbm;

extern "C" {

int evlbm_init_slab(evlbm_t h, double x0, double x1, double Tr, double width, uint64_t seed, double noise)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    if (!(Tr > 0) || !(width > 0) || !(noise >= 0 && noise < 1) || !(x1 > x0))
        return fail(EVLBM_EINVAL, "bad slab arguments (T/Tc, width > 0, 0 <= noise < 1, x1 > x0)");
    double cp[3], co[3];
    int rc = coexistence_at(h, Tr, cp, co);
    if (rc) return rc;
    double *d = nullptr;
    rc = two_fields(h, &d);
    if (rc) return rc;
    const long N = h->N;
    hipLaunchKernelGGL(k_slab, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, h->stream, h->nx, N, x0, x1, width,
                       co[0], co[1], Tr * cp[1], seed, noise, d, d + N);
    hipError_t e = hipGetLastError();
    rc = e == hipSuccess ? evlbm_init_fields(h, d, nullptr, d + N, EVLBM_DEVICE_F64) : hip_fail(e, "slab fields");
    (void)hipFree(d);
    return rc;
}

int evlbm_init_droplet(evlbm_t h, double cx, double cy, double cz, double R, double Tr, int profile, evlbm_mlp_t mlp,
                       double width, uint64_t seed, double noise, int *used_mlp)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    double *d = nullptr;
    int rc = two_fields(h, &d);
    if (rc) return rc;
    bool used = false;
    rc = droplet_fields(h, cx, cy, cz, R, Tr, profile, mlp, width, seed, noise, d, d + h->N, &used);
    if (rc == EVLBM_OK) rc = evlbm_init_fields(h, d, nullptr, d + h->N, EVLBM_DEVICE_F64);
    (void)hipFree(d);
    if (rc == EVLBM_OK && used_mlp) *used_mlp = used ? 1 : 0;
    return rc;
}

int evlbm_init_droplet_matched(evlbm_t h, double cx, double cy, double cz, double R, double Tr, int profile,
                               evlbm_mlp_t mlp, double width, uint64_t seed, double noise, double mass,
                               double energy, int *used_mlp, double *T_used)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    if (!(mass > 0) || !std::isfinite(energy)) return fail(EVLBM_EINVAL, "need mass > 0 and a finite energy");
    double *d = nullptr;
    int rc = two_fields(h, &d);
    if (rc) return rc;
    const long N = h->N;
    const unsigned nb = (unsigned)((N + 255) / 256);
    bool used = false;
    double s[8], T1 = 0.0;
    rc = droplet_fields(h, cx, cy, cz, R, Tr, profile, mlp, width, seed, noise, d, d + N, &used);
    double cp[3] = {0.0, 0.0, 0.0}, co[3] = {0.0, 0.0, 0.0};
    if (rc == EVLBM_OK) rc = coexistence_at(h, Tr, cp, co);
    const double T0 = Tr * cp[1];
    // the stored mass of the profile, then the profile scaled to `mass`
    if (rc == EVLBM_OK) rc = evlbm_init_fields(h, d, nullptr, d + N, EVLBM_DEVICE_F64);
    if (rc == EVLBM_OK) rc = evlbm_global_sums(h, s);
    if (rc == EVLBM_OK) {
        hipLaunchKernelGGL(k_noise_scale, dim3(nb), dim3(256), 0, h->stream, d, d + N, N, seed, 0.0, mass / s[0], T0);
        rc = evlbm_init_fields(h, d, nullptr, d + N, EVLBM_DEVICE_F64);
    }
    // At rest and uniform T the total energy (global sum 5) grows by (3/2) R M
    // per unit of T, up to the weak dependence of the streamed density (and
    // so of the force terms) on theta: Newton steps on T with that slope
    // until the energy agrees to 1e-13 (at most 8).
    T1 = T0;
    for (int it = 0; it < 8 && rc == EVLBM_OK; ++it) {
        rc = evlbm_global_sums(h, s);
        if (rc) break;
        const double dT = (energy - s[5]) / (1.5 * h->R * mass);
        if (std::fabs(energy - s[5]) <= 1e-13 * std::fabs(energy)) break;
        T1 += dT;
        if (!(T1 > 0)) {
            rc = fail(EVLBM_ENONPHYS, "no positive temperature gives the requested energy");
            break;
        }
        hipLaunchKernelGGL(k_noise_scale, dim3(nb), dim3(256), 0, h->stream, d, d + N, N, seed, 0.0, 1.0, T1);
        rc = evlbm_init_fields(h, d, nullptr, d + N, EVLBM_DEVICE_F64);
    }
    (void)hipFree(d);
    if (rc == EVLBM_OK) {
        if (used_mlp) *used_mlp = used ? 1 : 0;
        if (T_used) *T_used = T1;
    }
    return rc;
}

}  // extern "C"
