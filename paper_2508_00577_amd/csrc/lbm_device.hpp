// Device-side building blocks of the Enskog-Vlasov lattice Boltzmann step
// (Karlin & Hosseini, arXiv 2508.00577) for gfx950: lattice constants,
// 16-bit deviation codecs, isotropic stencils on LDS tiles and the per-axis
// factors of the product equilibria.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "evlbm.h"

namespace evlbm {

template <int D>
struct Lat {
    static constexpr int Q = (D == 2) ? 9 : 27;
    static constexpr int HZ = (D == 3) ? 1 : 0;  // 1 where the z direction exists
};

// Velocity index i = (cx+1) + 3 (cy+1) + 9 (cz+1) on D3Q27; D2Q9 uses the
// first nine indices i = (cx+1) + 3 (cy+1) with cz = 0.
__host__ __device__ constexpr int cx_of(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy_of(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz_of(int i) { return (i / 9) % 3 - 1; }
template <int D>
__host__ __device__ constexpr int cz_d(int i) { return D == 3 ? cz_of(i) : 0; }

// 1D lattice weights: 2/3 for c = 0, 1/6 for c = +-1 (their products are the
// D2Q9 / D3Q27 weights).
template <typename R>
__host__ __device__ constexpr R w1(int c) { return c == 0 ? R(2) / R(3) : R(1) / R(6); }

__host__ __device__ inline int wrapi(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

// ------------------------------------------------------------------ codecs

// gfx950 converts in hardware (v_cvt_pk_bf16_f32): round to nearest even,
// NaN stays NaN.
__device__ inline uint16_t f32_to_bf16_rne(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ inline uint16_t f32_to_f16_rne(float v)
{
    _Float16 h = (_Float16)v;  // v_cvt_f16_f32 rounds to nearest even
    return __builtin_bit_cast(uint16_t, h);
}

__device__ inline float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// Reference of a stored population (16-bit deviation storage): value r, a
// positive scale s of the population's magnitude and, where the population
// is encoded, is ~ 1/s; the stored quantity is the scaled deviation
// (v - r) is, decoded as r + s h, so its 16 bits resolve the deviation
// relative to the population itself (FP16 keeps it in its normal range even
// for the smallest diagonal populations).  Unused ({0, 1, 1}) by the plain
// storages.
template <typename R>
struct Ref {
    R r, s, is;
};

// Reciprocal for the per-cell 1/rho and 1/(1 - b rho): the hardware
// approximation (<= 1 ulp) in FP32, an exact division in FP64.
template <typename R>
__device__ inline R rcp(R x)
{
    if constexpr (sizeof(R) == 4)
        return __builtin_amdgcn_rcpf(x);
    else
        return R(1) / x;
}

// Storage traits: T = stored type, R = arithmetic type.
template <int S>
struct Codec;

template <>
struct Codec<EVLBM_F64> {
    using T = double;
    using R = double;
    static __device__ inline R dec(T v, Ref<R>) { return v; }
    static __device__ inline T enc(R v, Ref<R>) { return v; }
};

template <>
struct Codec<EVLBM_F32> {
    using T = float;
    using R = float;
    static __device__ inline R dec(T v, Ref<R>) { return v; }
    static __device__ inline T enc(R v, Ref<R>) { return v; }
};

// 16-bit decodes are one explicit fused multiply-add: whether the compiler
// fuses r + s h on its own depends on the surrounding code, and a stored value
// must decode to the same bits in every kernel that pulls it (the one-pass and
// two-pass steps agree bit for bit).
template <>
struct Codec<EVLBM_F16DEV> {
    using T = uint16_t;
    using R = float;
    static __device__ inline R dec(T v, Ref<R> q) { return __builtin_fmaf(q.s, f16_to_f32(v), q.r); }
    static __device__ inline T enc(R v, Ref<R> q) { return f32_to_f16_rne((v - q.r) * q.is); }
};

template <>
struct Codec<EVLBM_BF16DEV> {
    using T = uint16_t;
    using R = float;
    static __device__ inline R dec(T v, Ref<R> q) { return __builtin_fmaf(q.s, bf16_to_f32(v), q.r); }
    static __device__ inline T enc(R v, Ref<R> q) { return f32_to_bf16_rne((v - q.r) * q.is); }
};

// ------------------------------------------------------------ parameters

template <typename R>
struct StepParams {
    int nx, ny, nz;
    long N;          // cells
    long ds;         // elements between consecutive direction arrays of the populations (>= N)
    int eos;         // contact factor of Enskog's pressure: EVLBM_EOS_VDW or EVLBM_EOS_CS (enskog())
    R a, b, kappa;   // EOS: P_E = rho RT Z(rho) (b: excluded volume), P_V = -a rho^2, capillarity
    R two_beta;      // 2 beta, beta = 1/(2 tau + 1)
    R wstar;         // (dt/lambda)(1 - beta)
    R two_beta_g;    // the same for the energy populations, beta_g = 1/(2 tau/Pr + 1)
    R wstar_g;       // (dt/lambda)(1 - beta_g)
    R qe;            // 2 (beta_g - beta): weight of the quasi-equilibrium flux term (0 at Pr = 1)
    int vpr;         // 1 when Pr != 1 (the quasi-equilibrium pre-pass runs)
    R lambda, sphi;
    R Rgas;
    const float4 *refst;  // 16-bit deviation storage: reference state of every cell (ref_state_of)
};

// ---------------------------------------------------- Enskog pressure

// Enskog's pressure P_E = rho R T (1 + b rho chi) = rho R T Z(rho) with the
// contact value chi of the pair distribution (the text after eq. Ework):
//   EVLBM_EOS_VDW  chi = 1/(1 - b rho):  Z = 1/(1 - b rho) (the paper's form)
//   EVLBM_EOS_CS   chi = (1 - eta/2)/(1 - eta)^3, eta = b rho/4 (Carnahan-
//                  Starling): Z = (1 + eta + eta^2 - eta^3)/(1 - eta)^3.
// Under the gauge P0 = P_E (eq. P0E), theta = P0/rho = RT Z and eq. gamma
// gives gamma_0 = 1 + d ln Z/d ln rho + (2/3) Z, so the factor of
// eq. correction_gamma is 5/3 - gamma_0:
//   van der Waals: (5/3)(1 - Z);
//   Carnahan-Starling: 2/3 - (2/3) Z - d ln Z/d ln rho with
//   d ln Z/d ln rho = eta (1 + 2 eta - 3 eta^2)/(1 + eta + eta^2 - eta^3) + 3 eta/(1 - eta).
template <typename R>
struct Enskog {
    R Z;   // P_E/(rho R T)
    R g5;  // 5/3 - gamma_0
};

template <typename R>
__device__ inline Enskog<R> enskog(int eos, R b, R rho)
{
    if (eos == EVLBM_EOS_CS) {
        const R eta = R(0.25) * b * rho;
        const R i1 = rcp(R(1) - eta);
        const R num = R(1) + eta * (R(1) + eta * (R(1) - eta));
        const R Z = num * (i1 * i1 * i1);
        const R dlnZ = eta * (R(1) + eta * (R(2) - R(3) * eta)) * rcp(num) + R(3) * eta * i1;
        return Enskog<R>{Z, (R(2) / R(3)) * (R(1) - Z) - dlnZ};
    }
    const R Z = rcp(R(1) - b * rho);
    return Enskog<R>{Z, (R(5) / R(3)) * (R(1) - Z)};
}

// The same with the closure fixed at compile time (EOSK = EVLBM_EOS_VDW or
// EVLBM_EOS_CS) or, for EOSK < 0, taken from eos at run time.
template <int EOSK, typename R>
__device__ inline Enskog<R> enskog_k(int eos, R b, R rho)
{
    return enskog<R>(EOSK < 0 ? eos : EOSK, b, rho);
}

// FP64 form for initialisation, validation and measurement (exact divisions);
// false outside the closure's range (b rho >= 1, resp. eta >= 1).
__host__ __device__ inline bool enskog_z64(int eos, double b, double rho, double *Z)
{
    if (eos == EVLBM_EOS_CS) {
        const double eta = 0.25 * b * rho;
        if (!(eta < 1.0)) return false;
        *Z = (1.0 + eta + eta * eta - eta * eta * eta) / ((1.0 - eta) * (1.0 - eta) * (1.0 - eta));
        return true;
    }
    if (!(1.0 - b * rho > 0.0)) return false;
    *Z = 1.0 / (1.0 - b * rho);
    return true;
}

// ------------------------------------------------------------ addressing

// Every direction array of a lattice holds N cells and is below 4 GiB (the
// host rejects larger lattices), so a cell is addressed by a uniform 64-bit
// base (the direction's array, kept in scalar registers) plus a 32-bit byte
// offset: one vector register per address and the saddr + voffset form of
// the global loads and stores.
template <typename T>
__device__ inline T ld_at(const T *__restrict__ base, unsigned byte)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte);
}

// Stores of 4- and 8-byte elements are non-temporal: the step's outputs are
// not re-read before the next launch, so they bypass the caches instead of
// evicting reused lines.  16-bit elements are stored normally so the L2 can
// merge them into full lines.
template <typename T>
__device__ inline void st_at(T *__restrict__ base, unsigned byte, T v)
{
    T *q = reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte);
    if constexpr (sizeof(T) >= 4)
        __builtin_nontemporal_store(v, q);
    else
        *q = v;
}


// Population access through per-direction pointers: array p (0..2Q-1: f
// directions, then g) of src or dst at a byte offset.
template <typename T>
struct PtrPops {
    const T *src;
    T *dst;
    long ds;  // direction stride (elements)
    __device__ inline T ld(int pop, unsigned byte) const { return ld_at(src + (long)pop * ds, byte); }
    __device__ inline void st(int pop, unsigned byte, T v) const { st_at(dst + (long)pop * ds, byte, v); }
};

// Population access through raw buffer resources: one resource per
// population (f, g) of src and dst, the direction's offset i * ds * sizeof(T)
// in a scalar register shared by all four, the cell's byte offset in a vector
// register.  This keeps the 4Q per-direction base pointers of a D3Q27 step
// out of the scalar register file, which otherwise spills them to vector
// lanes.  Valid while Q * ds * sizeof(T) < 2^32 (the launcher checks), so
// that every offset sum stays below 2^32.
constexpr int RSRC_WORD3 = 0x00020000;  // raw (untyped) buffer, 32-bit data, gfx9 family

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1, RSRC_WORD3);
}

template <typename T>
__device__ inline T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    if constexpr (sizeof(T) == 2)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0));
    else if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

// Stores of 4- and 8-byte elements carry the non-temporal hint (cache policy
// bit 1), as st_at does.
template <typename T>
__device__ inline void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, T v)
{
    if constexpr (sizeof(T) == 2)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)voff, (int)soff, 0);
    else if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 2);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                              (int)voff, (int)soff, 2);
}

template <typename T, int Q>
struct BufPops {
    __amdgpu_buffer_rsrc_t sf, sg, df, dg;
    unsigned dir;  // bytes between consecutive direction arrays: ds * sizeof(T)
    __device__ inline BufPops(const T *src, T *dst, long ds)
        : sf(make_rsrc(src)), sg(make_rsrc(src + (long)Q * ds)), df(make_rsrc(dst)), dg(make_rsrc(dst + (long)Q * ds)),
          dir((unsigned)ds * (unsigned)sizeof(T))
    {
    }
    __device__ inline T ld(int pop, unsigned byte) const
    {
        return pop < Q ? buf_ld<T>(sf, byte, (unsigned)pop * dir) : buf_ld<T>(sg, byte, (unsigned)(pop - Q) * dir);
    }
    __device__ inline void st(int pop, unsigned byte, T v) const
    {
        if (pop < Q)
            buf_st<T>(df, byte, (unsigned)pop * dir, v);
        else
            buf_st<T>(dg, byte, (unsigned)(pop - Q) * dir, v);
    }
};

// Byte offsets of the pull sources of a cell in arrays of ES-byte elements:
// entry k = c + 1 of each axis holds the periodic source coordinate x - c,
// so direction i reads ox[cx+1] + oy[cy+1] + oz[cz+1].
struct PullOffsets {
    unsigned ox[3], oy[3], oz[3];
};

template <int D, int ES>
__device__ inline PullOffsets pull_offsets(int nx, int ny, int nz, int x, int y, int z)
{
    PullOffsets o;
    const unsigned sy = (unsigned)nx * ES, sz = (unsigned)nx * (unsigned)ny * ES;
    o.ox[0] = (unsigned)(x + 1 == nx ? 0 : x + 1) * ES;
    o.ox[1] = (unsigned)x * ES;
    o.ox[2] = (unsigned)(x == 0 ? nx - 1 : x - 1) * ES;
    o.oy[0] = (unsigned)(y + 1 == ny ? 0 : y + 1) * sy;
    o.oy[1] = (unsigned)y * sy;
    o.oy[2] = (unsigned)(y == 0 ? ny - 1 : y - 1) * sy;
    if (D == 3) {
        o.oz[0] = (unsigned)(z + 1 == nz ? 0 : z + 1) * sz;
        o.oz[1] = (unsigned)z * sz;
        o.oz[2] = (unsigned)(z == 0 ? nz - 1 : z - 1) * sz;
    } else {
        o.oz[0] = o.oz[1] = o.oz[2] = 0u;
    }
    return o;
}

// Reference of the 16-bit deviation storage: the equilibrium at rest of a
// per-cell reference state (rho, theta = RT/(1 - b rho), K = (3/2) RT).  At
// u = 0 the product equilibrium (eq. feq) is rho prod_a psi(c_a; 0, theta)
// with psi(0) = w0 = 1 - theta and psi(+-1) = w1 = theta/2, so for
// n = |c_i|^2 it is a0 q^n with a0 = rho w0^D and q = w1/w0; the energy
// equilibrium (eq. geq) is f^eq_i [K + n theta - (D - n) theta^2/(1 - theta)]
// = f^eq_i (A + n B) with A = K - D theta^2/(1 - theta) and B =
// theta/(1 - theta) (O A = 0 and O^2 A = theta^2 at rest: the factors
// chi(0) = -theta^2 and chi(+-1) = theta^2/2 divided by psi).  A cell stores
// the state as {a0, q, A, B}; scales are f^eq for f and B f^eq for g (both
// positive).
template <int D, typename V = double>
__host__ __device__ inline float4 ref_state_of(V rho, V theta, V K)
{
    const V w0 = V(1) - theta, w1 = V(0.5) * theta;
    V a0 = rho;
    for (int k = 0; k < D; ++k) a0 *= w0;
    return make_float4((float)a0, (float)(w1 / w0), (float)(K - V(D) * theta * theta / w0), (float)(theta / w0));
}

// Reference value and scale of population pop (f 0..Q-1, then g) for a cell
// with reference state rs (decode side: is left 0).
template <int D, typename R>
__device__ inline Ref<R> ref_value(int pop, float4 rs)
{
    constexpr int Q = Lat<D>::Q;
    const int i = pop < Q ? pop : pop - Q;
    const int n = cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_d<D>(i) * cz_d<D>(i);
    static_assert(sizeof(R) == 4, "16-bit storage decodes in FP32");
    R f = (R)rs.x;
    for (int k = 0; k < n; ++k) f *= (R)rs.y;
    if (pop < Q) return Ref<R>{f, f, R(0)};
    // A + n B as one explicit fused multiply-add (see the 16-bit codecs)
    return Ref<R>{f * __builtin_fmaf(R(n), (R)rs.w, (R)rs.z), f * (R)rs.w, R(0)};
}

// The reciprocals an encoding cell needs, computed once per cell.
template <typename R>
struct RefInv {
    R ia0, iq, iB;
};

template <typename R>
__device__ inline RefInv<R> ref_inv(float4 rs)
{
    return RefInv<R>{rcp((R)rs.x), rcp((R)rs.y), rcp((R)rs.w)};
}

// Encode side: the reference with is = 1/s from the cell's reciprocals.
template <int D, typename R>
__device__ inline Ref<R> ref_value_enc(int pop, float4 rs, RefInv<R> v)
{
    constexpr int Q = Lat<D>::Q;
    Ref<R> q = ref_value<D, R>(pop, rs);
    const int i = pop < Q ? pop : pop - Q;
    const int n = cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_d<D>(i) * cz_d<D>(i);
    R is = v.ia0;
    for (int k = 0; k < n; ++k) is *= v.iq;
    q.is = pop < Q ? is : is * v.iB;
    return q;
}

// Reference state of the cell at element index s / 16-bit byte offset byte16.
template <int S, typename R>
__device__ inline float4 ref_state_at(const StepParams<R> &p, long s)
{
    if constexpr (S == EVLBM_F16DEV || S == EVLBM_BF16DEV)
        return p.refst[s];
    else
        return make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int S, typename R>
__device__ inline float4 ref_state_at_b(const StepParams<R> &p, unsigned byte16)
{
    if constexpr (S == EVLBM_F16DEV || S == EVLBM_BF16DEV)
        return ld_at(p.refst, byte16 * 8u);
    else
        return make_float4(0.f, 0.f, 0.f, 0.f);
}

// Decode-side reference of population pop stored at cell s (element index)
// or at 16-bit byte offset byte16; {0, 1, 1} for the plain storages.
template <int D, int S, typename R>
__device__ inline Ref<R> ref_at(const StepParams<R> &p, int pop, long s)
{
    if constexpr (S == EVLBM_F16DEV || S == EVLBM_BF16DEV)
        return ref_value<D, R>(pop, p.refst[s]);
    else
        return Ref<R>{R(0), R(1), R(1)};
}

template <int D, int S, typename R>
__device__ inline Ref<R> ref_at_b(const StepParams<R> &p, int pop, unsigned byte16)
{
    if constexpr (S == EVLBM_F16DEV || S == EVLBM_BF16DEV)
        return ref_value<D, R>(pop, ld_at(p.refst, byte16 * 8u));
    else
        return Ref<R>{R(0), R(1), R(1)};
}

// Encode-side reference of population pop of a cell whose state rs and
// reciprocals inv were loaded once.
template <int D, int S, typename R>
__device__ inline Ref<R> ref_enc(int pop, float4 rs, RefInv<R> inv)
{
    if constexpr (S == EVLBM_F16DEV || S == EVLBM_BF16DEV)
        return ref_value_enc<D, R>(pop, rs, inv);
    else
        return Ref<R>{R(0), R(1), R(1)};
}

template <int S, typename R>
__device__ inline RefInv<R> ref_inv_of(float4 rs)
{
    if constexpr (S == EVLBM_F16DEV || S == EVLBM_BF16DEV)
        return ref_inv<R>(rs);
    else
        return RefInv<R>{R(1), R(1), R(1)};
}

// ---------------------------------------------- per-axis equilibrium factors

// psi(c; xi, zeta) of eq. phi, indexed by k = c + 1:
// psi(0) = 1 - zeta, psi(+-1) = (zeta +- xi)/2.
template <typename R>
__device__ inline void psi3(R xi, R zeta, R out[3])
{
    out[0] = R(0.5) * (zeta - xi);
    out[1] = R(1) - zeta;
    out[2] = R(0.5) * (zeta + xi);
}

// Operator factors of the energy equilibrium (eq. geq) on A = u^2/2 with
// O A = theta dA/du + u A:  O A = theta u + u^3/2,
// O^2 A = theta^2 + (5/2) theta u^2 + u^4/2;  chi(0) = A - O^2 A,
// chi(+-1) = (O^2 A +- O A)/2.  With phi = psi(c; u, theta + u^2):
// g_i = rho [ (3/2) RT prod_a phi_a + sum_b chi_b prod_{a != b} phi_a ].
template <typename R>
__device__ inline void chi3(R u, R theta, R out[3])
{
    R u2 = u * u;
    R A = R(0.5) * u2;
    R OA = theta * u + R(0.5) * u2 * u;
    R O2A = theta * theta + R(2.5) * theta * u2 + R(0.5) * u2 * u2;
    out[0] = R(0.5) * (O2A - OA);
    out[1] = A - O2A;
    out[2] = R(0.5) * (O2A + OA);
}

// ------------------------------------------------- isotropic LDS stencils

// d_a phi = 3 sum_i w_i c_ia phi(x + c_i) on an LDS box with strides (1, sy, sz).
template <int D, int A, typename R>
__device__ inline R lds_grad(const R *s, int c, int sy, int sz)
{
    constexpr int HZ = Lat<D>::HZ;
    R acc = R(0);
#pragma unroll
    for (int dz = -HZ; dz <= HZ; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int ca = (A == 0) ? dx : (A == 1) ? dy : dz;
                if (ca == 0) continue;
                const R w = w1<R>(dx) * w1<R>(dy) * (D == 3 ? w1<R>(dz) : R(1));
                acc += (R(3) * w * R(ca)) * s[c + dx + dy * sy + dz * sz];
            }
    return acc;
}

// lap phi = 6 sum_i w_i (phi(x + c_i) - phi(x)).
template <int D, typename R>
__device__ inline R lds_lap(const R *s, int c, int sy, int sz)
{
    constexpr int HZ = Lat<D>::HZ;
    R acc = R(0);
    const R centre = s[c];
#pragma unroll
    for (int dz = -HZ; dz <= HZ; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const R w = w1<R>(dx) * w1<R>(dy) * (D == 3 ? w1<R>(dz) : R(1));
                acc += (R(6) * w) * (s[c + dx + dy * sy + dz * sz] - centre);
            }
    return acc;
}

// Gradient of rho^2 from an LDS box of rho (the conservative mean-field force).
template <int D, int A, typename R>
__device__ inline R lds_grad_sq(const R *s, int c, int sy, int sz)
{
    constexpr int HZ = Lat<D>::HZ;
    R acc = R(0);
#pragma unroll
    for (int dz = -HZ; dz <= HZ; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int ca = (A == 0) ? dx : (A == 1) ? dy : dz;
                if (ca == 0) continue;
                const R w = w1<R>(dx) * w1<R>(dy) * (D == 3 ? w1<R>(dz) : R(1));
                const R v = s[c + dx + dy * sy + dz * sz];
                acc += (R(3) * w * R(ca)) * (v * v);
            }
    return acc;
}

}  // namespace evlbm
