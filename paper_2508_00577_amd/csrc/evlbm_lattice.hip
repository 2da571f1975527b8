// C ABI of one periodic lattice (declared in include/evlbm.h): handle life
// cycle, parameters, initialisation, time stepping, readout, reductions,
// population I/O and checkpoints.
#include <cmath>
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "evlbm_internal.hpp"
#include "evlbm_params.hpp"
#include "lbm_kernels.hpp"

using namespace evlbm;

namespace evlbm {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(EVLBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t store_bytes(int storage) { return storage == EVLBM_F64 ? 8 : storage == EVLBM_F32 ? 4 : 2; }

// Bytes between the end of one population direction array and the start of
// the next (a multiple of 256 bytes, not of 4 KiB; measured best of 256 B to
// 48 KiB on the 256^3 D3Q27 FP32 step).
static constexpr long DIR_PAD = 1280;
size_t real_bytes(int storage) { return storage == EVLBM_F64 ? 8 : 4; }

template <typename R>
StepParams<R> make_params(const evlbm_lattice *h)
{
    StepParams<R> p = model_params<R>(h->eos, h->R, h->a, h->b, h->kappa, h->tau, h->lambda, h->sphi, h->prandtl);
    p.nx = h->nx;
    p.ny = h->ny;
    p.nz = h->nz;
    p.N = h->N;
    p.ds = h->ds;
    p.refst = h->refst;
    return p;
}

template StepParams<float> make_params<float>(const evlbm_lattice *);
template StepParams<double> make_params<double>(const evlbm_lattice *);

static dim3 row_grid(const evlbm_lattice *h, int bx) { return dim3((h->nx + bx - 1) / bx, h->ny, h->nz); }
static int row_block(const evlbm_lattice *h) { return h->nx >= 256 ? 256 : ((h->nx + 63) / 64) * 64; }

// ------------------------------------------------------------- dispatch

template <int D, int S>
struct Ops {
    using T = StoreT<S>;
    using R = RealT<S>;
    // tile of the collision kernel
    static constexpr int BX = (D == 2) ? 64 : (S == EVLBM_F64 ? 16 : 32);
    static constexpr int BY = (D == 2) ? 16 : 4;  // D2Q9: 64 x 16 measured best for the one-pass step
    static constexpr int BZ = (D == 2) ? 1 : 2;

    static void moments(evlbm_lattice *h, const void *pop)
    {
        const int bx = row_block(h);
        hipLaunchKernelGGL((k_moments<D, S>), row_grid(h, bx), dim3(bx), 0, h->stream, (const T *)pop, (R *)h->m,
                           make_params<R>(h));
    }
    // z-marching tile of the D3Q27 kernel: TX x TY columns, ZC planes per chunk
    // (64 x 4 in FP32 and 16-bit storage: a row of the tile spans two 128-byte
    // lines, so the pulled rows of the 18 directions with cx != 0 touch three)
    static constexpr int TX = (S == EVLBM_F64) ? 16 : 64;
    static constexpr int TY = (S == EVLBM_F64) ? 8 : 4;
    // planes per chunk, measured at 256^3: in FP32 40 is best of 32..64 (2.9 %
    // faster than 32); the FP64 tile (one wave per SIMD) gains up to 64
    static constexpr int ZC = (S == EVLBM_F64) ? 64 : 40;
    // the one-pass step (FP32 and FP64 storage: with 16-bit storage the
    // collision's registers leave no room for the pushed sums at 2 waves per SIMD)
    static constexpr bool PUSH_OK = D == 3 && (S == EVLBM_F32 || S == EVLBM_F64);
    static long shell_elems(const evlbm_lattice *h)
    {
        const long nb = (long)((h->nx + TX - 1) / TX) * ((h->ny + TY - 1) / TY) * ((h->nz + ZC - 1) / ZC);
        return nb * 5 * Shell<TX, TY, ZC>::SIZE;
    }

    template <bool PUSH>
    static void collide_zm(evlbm_lattice *h, const void *src, void *dst)
    {
        const int nbx = (h->nx + TX - 1) / TX, nby = (h->ny + TY - 1) / TY, nbz = (h->nz + ZC - 1) / ZC;
        R *mn = PUSH ? (R *)h->m_alt : nullptr, *sh = PUSH ? (R *)h->shell : nullptr;
        // buffer addressing while every offset into one population (f or g) stays below 2^32
        const bool buf = (double)27 * h->ds * sizeof(T) < 4294967296.0;
        const dim3 g(nbx * nby * nbz), b(TX, TY);
        if constexpr (!PUSH) {
            // Prandtl number != 1: the kernels with the quasi-equilibrium term
            if (h->prandtl != 1.0) {
                if (buf)
                    hipLaunchKernelGGL((k_collide_zm<S, TX, TY, ZC, true, false, true>), g, b, 0, h->stream,
                                       (const T *)src, (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, mn, sh);
                else
                    hipLaunchKernelGGL((k_collide_zm<S, TX, TY, ZC, false, false, true>), g, b, 0, h->stream,
                                       (const T *)src, (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, mn, sh);
                return;
            }
        }
        if constexpr (PUSH) {
            // the one-pass step, the benchmark's kernel: the pressure closure
            // is compiled in rather than branched on per cell, and so is the
            // quasi-equilibrium term of Pr != 1 (251 VGPRs with it, still two
            // waves per SIMD in FP32)
            const bool vpr = h->prandtl != 1.0;
            if (buf && h->eos == EVLBM_EOS_VDW && !vpr)
                hipLaunchKernelGGL((k_collide_zm<S, TX, TY, ZC, true, true, false, EVLBM_EOS_VDW>), g, b, 0, h->stream,
                                   (const T *)src, (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, mn, sh);
            else if (buf && !vpr)
                hipLaunchKernelGGL((k_collide_zm<S, TX, TY, ZC, true, true, false, EVLBM_EOS_CS>), g, b, 0, h->stream,
                                   (const T *)src, (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, mn, sh);
            else if (buf)
                hipLaunchKernelGGL((k_collide_zm<S, TX, TY, ZC, true, true, true>), g, b, 0, h->stream,
                                   (const T *)src, (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, mn, sh);
            else if (!vpr)
                hipLaunchKernelGGL((k_collide_zm<S, TX, TY, ZC, false, true>), g, b, 0, h->stream, (const T *)src,
                                   (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, mn, sh);
            else
                hipLaunchKernelGGL((k_collide_zm<S, TX, TY, ZC, false, true, true>), g, b, 0, h->stream,
                                   (const T *)src, (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, mn, sh);
            return;
        }
        if (buf)
            hipLaunchKernelGGL((k_collide_zm<S, TX, TY, ZC, true, PUSH>), g, b, 0, h->stream, (const T *)src, (T *)dst,
                               (const R *)h->m, make_params<R>(h), nbx, nby, mn, sh);
        else
            hipLaunchKernelGGL((k_collide_zm<S, TX, TY, ZC, false, PUSH>), g, b, 0, h->stream, (const T *)src, (T *)dst,
                               (const R *)h->m, make_params<R>(h), nbx, nby, mn, sh);
    }

    // D3Q27 one-pass step: collision pushing the next moments into m_alt and
    // the shell, then the fix-up that completes m_alt (event `between` is
    // recorded between the two when given)
    static void collide_push(evlbm_lattice *h, const void *src, void *dst, hipEvent_t between)
    {
        if constexpr (PUSH_OK) {
            collide_zm<true>(h, src, dst);
            if (between) (void)hipEventRecord(between, h->stream);
            const int nbx = (h->nx + TX - 1) / TX, nby = (h->ny + TY - 1) / TY, nbz = (h->nz + ZC - 1) / ZC;
            hipLaunchKernelGGL((k_push_fixup<R, TX, TY, ZC>), dim3(nbx * nby * nbz, ZC), dim3(TX, TY), 0, h->stream,
                               (R *)h->m_alt, (const R *)h->shell, h->nx, h->ny, h->nz, nbx, nby, nbz);
        }
    }

    static void collide(evlbm_lattice *h, const void *src, void *dst)
    {
        if constexpr (D == 3) {
            collide_zm<false>(h, src, dst);
        } else {
            // D2Q9: the one-pass step sums the moments of its halo from the
            // pulled populations in the collision itself (no moment pass)
            const int nbx = (h->nx + BX - 1) / BX, nby = (h->ny + BY - 1) / BY, nbz = (h->nz + BZ - 1) / BZ;
            const int nt = nbx * nby * nbz;
            if (h->prandtl != 1.0)
                hipLaunchKernelGGL((k_collide<D, S, BX, BY, BZ, true, true>), dim3(nt), dim3(BX, BY, BZ), 0, h->stream,
                                   (const T *)src, (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, nt);
            else if (h->push)
                hipLaunchKernelGGL((k_collide<D, S, BX, BY, BZ, true>), dim3(nt), dim3(BX, BY, BZ), 0, h->stream,
                                   (const T *)src, (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, nt);
            else
                hipLaunchKernelGGL((k_collide<D, S, BX, BY, BZ>), dim3(nt), dim3(BX, BY, BZ), 0, h->stream,
                                   (const T *)src, (T *)dst, (const R *)h->m, make_params<R>(h), nbx, nby, nt);
        }
    }
    static void init(evlbm_lattice *h, const double *rho, const double *u, const double *T0)
    {
        const long nb = (h->N + 255) / 256;
        hipLaunchKernelGGL((k_init<D, S>), dim3(nb), dim3(256), 0, h->stream, rho, u, T0, (T *)h->buf[h->cur],
                           make_params<R>(h));
    }
    static void lap(evlbm_lattice *h)
    {
        const int bx = row_block(h);
        hipLaunchKernelGGL((k_lap_field<D, R>), row_grid(h, bx), dim3(bx), 0, h->stream, (const R *)h->m, (R *)h->lap,
                           h->nx, h->ny, h->nz);
    }
    template <typename O>
    static void readout(evlbm_lattice *h, O *rho, O *u, O *T0)
    {
        const int bx = row_block(h);
        hipLaunchKernelGGL((k_readout<D, R, O>), row_grid(h, bx), dim3(bx), 0, h->stream, (const R *)h->m,
                           (const R *)h->lap, rho, u, T0, h->nx, h->ny, h->nz, (R)h->a, (R)h->kappa, (R)h->R);
    }
    static void sums(evlbm_lattice *h, double *partial, long nb)
    {
        hipLaunchKernelGGL((k_sums<D, S>), dim3(nb), dim3(256), 0, h->stream, (const T *)h->buf[h->cur],
                           (const R *)h->m, (const R *)h->lap, make_params<R>(h), partial);
    }
    static void measure(evlbm_lattice *h, int kind, const double *g, double *partial, long nb)
    {
        hipLaunchKernelGGL((k_measure<D, R>), dim3(nb), dim3(256), 0, h->stream, (const R *)h->m, (const R *)h->lap,
                           h->nx, h->ny, h->nz, h->eos, (R)h->a, (R)h->b, (R)h->kappa, (R)h->R, kind, g[0], g[1], g[2], g[3],
                           g[4], g[5], partial);
    }
    static void decode(evlbm_lattice *h, double *out)
    {
        const long n = h->N * 2 * h->Q;
        hipLaunchKernelGGL((k_decode<D, S>), dim3((n + 255) / 256), dim3(256), 0, h->stream, (const T *)h->buf[h->cur],
                           out, h->N, 2 * h->Q, make_params<R>(h));
    }
    static void encode(evlbm_lattice *h, const double *in)
    {
        const long n = h->N * 2 * h->Q;
        hipLaunchKernelGGL((k_encode<D, S>), dim3((n + 255) / 256), dim3(256), 0, h->stream, in, (T *)h->buf[h->cur],
                           h->N, 2 * h->Q, make_params<R>(h));
    }
    static void rereference(evlbm_lattice *h)
    {
        if constexpr (S == EVLBM_F16DEV || S == EVLBM_BF16DEV)
            hipLaunchKernelGGL((k_rereference<D, S>), dim3((h->N + 255) / 256), dim3(256), 0, h->stream,
                               (T *)h->buf[h->cur], h->refst, make_params<R>(h));
    }
    static void ref_from_pops(evlbm_lattice *h, const double *pops)
    {
        hipLaunchKernelGGL((k_ref_from_pops<D>), dim3((h->N + 255) / 256), dim3(256), 0, h->stream, pops, h->N,
                           h->eos, h->b, h->refst);
    }
    static void scan(evlbm_lattice *h, int *flag)
    {
        hipLaunchKernelGGL((k_scan_nonfinite<R>), dim3((h->N + 255) / 256), dim3(256), 0, h->stream, (const R *)h->m,
                           h->N, flag);
    }
};

template <template <int, int> class F, typename... A>
static void dispatch(evlbm_lattice *h, A &&...args)
{
#define EVLBM_CASE(DD, SS) \
    if (h->D == DD && h->storage == SS) return F<DD, SS>::run(h, args...);
    EVLBM_CASE(2, EVLBM_F64)
    EVLBM_CASE(2, EVLBM_F32)
    EVLBM_CASE(2, EVLBM_F16DEV)
    EVLBM_CASE(2, EVLBM_BF16DEV)
    EVLBM_CASE(3, EVLBM_F64)
    EVLBM_CASE(3, EVLBM_F32)
    EVLBM_CASE(3, EVLBM_F16DEV)
    EVLBM_CASE(3, EVLBM_BF16DEV)
#undef EVLBM_CASE
}

template <int D, int S>
struct RunMoments {
    static void run(evlbm_lattice *h, const void *pop) { Ops<D, S>::moments(h, pop); }
};
template <int D, int S>
struct RunCollide {
    static void run(evlbm_lattice *h, const void *src, void *dst) { Ops<D, S>::collide(h, src, dst); }
};
template <int D, int S>
struct RunCollidePush {
    static void run(evlbm_lattice *h, const void *src, void *dst, hipEvent_t ev)
    {
        Ops<D, S>::collide_push(h, src, dst, ev);
    }
};
template <int D, int S>
struct RunShellElems {
    static void run(evlbm_lattice *h, long *n) { *n = Ops<D, S>::PUSH_OK ? Ops<D, S>::shell_elems(h) : 0; }
};
template <int D, int S>
struct RunInit {
    static void run(evlbm_lattice *h, const double *r, const double *u, const double *t) { Ops<D, S>::init(h, r, u, t); }
};
template <int D, int S>
struct RunLap {
    static void run(evlbm_lattice *h) { Ops<D, S>::lap(h); }
};
template <int D, int S>
struct RunReadoutF {
    static void run(evlbm_lattice *h, float *r, float *u, float *t) { Ops<D, S>::template readout<float>(h, r, u, t); }
};
template <int D, int S>
struct RunReadoutD {
    static void run(evlbm_lattice *h, double *r, double *u, double *t) { Ops<D, S>::template readout<double>(h, r, u, t); }
};
template <int D, int S>
struct RunSums {
    static void run(evlbm_lattice *h, double *p, long nb) { Ops<D, S>::sums(h, p, nb); }
};
template <int D, int S>
struct RunMeasure {
    static void run(evlbm_lattice *h, int kind, const double *g, double *p, long nb) { Ops<D, S>::measure(h, kind, g, p, nb); }
};
template <int D, int S>
struct RunDecode {
    static void run(evlbm_lattice *h, double *o) { Ops<D, S>::decode(h, o); }
};
template <int D, int S>
struct RunEncode {
    static void run(evlbm_lattice *h, const double *i) { Ops<D, S>::encode(h, i); }
};
template <int D, int S>
struct RunReref {
    static void run(evlbm_lattice *h) { Ops<D, S>::rereference(h); }
};
template <int D, int S>
struct RunRefFromPops {
    static void run(evlbm_lattice *h, const double *pops) { Ops<D, S>::ref_from_pops(h, pops); }
};
template <int D, int S>
struct RunScan {
    static void run(evlbm_lattice *h, int *f) { Ops<D, S>::scan(h, f); }
};

// ------------------------------------------------------------- helpers

int ensure_scratch(evlbm_lattice *h, size_t bytes)
{
    if (h->scratch_bytes >= bytes) return EVLBM_OK;
    if (h->scratch) hipFree(h->scratch);
    h->scratch = nullptr;
    h->scratch_bytes = 0;
    hipError_t e = hipMalloc(&h->scratch, bytes);
    if (e != hipSuccess) return fail(EVLBM_ENOMEM, "hipMalloc(%zu) for scratch: %s", bytes, hipGetErrorString(e));
    h->scratch_bytes = bytes;
    return EVLBM_OK;
}

// Make sure h->m holds the pulled moments of the current buffer (with walls:
// always pulled again, with the walls' re-emission).
void refresh_moments(evlbm_lattice *h)
{
    if (h->walls) {
        wall_analyse(h);
        h->m_valid = false;
        return;
    }
    if (!h->m_valid) {
        dispatch<RunMoments>(h, (const void *)h->buf[h->cur]);
        h->m_valid = true;
    }
}

static int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return EVLBM_OK;
}

// Run the reduction with NV values per block through the partial buffer;
// result copied to host out[NV].
static int finish_reduce(evlbm_lattice *h, long nb, int nv, const int ops[8], double *out)
{
    double *partial = (double *)h->scratch;
    double *res = partial + nb * nv;
    int4 lo = make_int4(ops[0], ops[1], ops[2], ops[3]);
    int4 hi = make_int4(ops[4], ops[5], ops[6], ops[7]);
    hipLaunchKernelGGL(k_reduce_final, dim3(nv), dim3(256), 0, h->stream, partial, nb, lo, hi, res);
    int rc = check_launch("reduce");
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(out, res, sizeof(double) * nv, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return EVLBM_OK;
}

int scan_nonfinite(evlbm_lattice *h)
{
    refresh_moments(h);
    int rc = ensure_scratch(h, sizeof(int) * 64);
    if (rc) return rc;
    int *flag = (int *)h->scratch;
    // clear with a copy (no memset node ever enters a captured graph here)
    int zero = 0;
    hipError_t e = hipMemcpyAsync(flag, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    dispatch<RunScan>(h, flag);
    int host = 0;
    e = hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (host) return fail(EVLBM_ENONFINITE, "%d cells with a non-finite or non-positive density at step %lld", host,
                          (long long)h->step);
    return EVLBM_OK;
}

// Does the step push the next moments (D3Q27 one-pass step)?
static bool pushes(const evlbm_lattice *h)
{
    return h->D == 3 && h->push && h->shell != nullptr && !h->walls;
}
// the one-pass D2Q9 step: the collision sums its halo's moments itself
static bool fused(const evlbm_lattice *h) { return h->D == 2 && h->push && !h->walls; }

// One step: moments of the current buffer, collision into the other.  The
// one-pass D3Q27 step also leaves the moments of the new state in m_alt,
// which becomes m; the one-pass D2Q9 step needs no moments.
void launch_step(evlbm_lattice *h, hipEvent_t between)
{
    if (h->walls) {
        if (between) (void)hipEventRecord(between, h->stream);
        wall_step(h);
        h->m_valid = false;
        h->cur = 1 - h->cur;
        h->step++;
        return;
    }
    if (!fused(h)) refresh_moments(h);
    const int nxt = 1 - h->cur;
    if (pushes(h)) {
        dispatch<RunCollidePush>(h, (const void *)h->buf[h->cur], h->buf[nxt], between);
        std::swap(h->m, h->m_alt);
        h->m_valid = true;
    } else {
        if (between) (void)hipEventRecord(between, h->stream);
        dispatch<RunCollide>(h, (const void *)h->buf[h->cur], h->buf[nxt]);
        h->m_valid = false;
    }
    h->cur = nxt;
    h->step++;
}

// 16-bit deviation storage: decode every cell's stored values with its
// reference state, take the state they carry (rho, theta) as the new
// reference and encode again, in place.
int rereference(evlbm_lattice *h)
{
    if (!h->refst) return EVLBM_OK;
    dispatch<RunReref>(h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "re-reference");
    h->m_valid = false;
    return EVLBM_OK;
}

// Steps are replayed from a captured graph of GRAPH_STEPS launches pairs
// (an even count, so the buffer parity is unchanged), one graph per parity.
static constexpr int GRAPH_STEPS = 32;

int run_steps(evlbm_lattice *h, int64_t n)
{
    const bool graph_ok = h->use_graph && h->stream != nullptr && n >= GRAPH_STEPS;
    if (!graph_ok) {
        for (int64_t k = 0; k < n; ++k) launch_step(h);
        return EVLBM_OK;
    }
    const int par = h->cur;
    // The one-pass step keeps the moments current, so its graph starts from
    // valid moments; the two-pass graph computes them itself.
    const bool push = pushes(h);
    if (push) refresh_moments(h);
    if (!h->graph_exec_par[par]) {
        const int cur0 = h->cur;
        const int64_t step0 = h->step;
        h->m_valid = push;
        hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        for (int k = 0; k < GRAPH_STEPS; ++k) launch_step(h);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(h->stream, &g);
        h->cur = cur0;
        h->step = step0;
        h->m_valid = push;
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        h->graph_exec_par[par] = ex;
    }
    const int64_t reps = n / GRAPH_STEPS;
    for (int64_t r = 0; r < reps; ++r) {
        hipError_t e = hipGraphLaunch(h->graph_exec_par[par], h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    h->step += reps * GRAPH_STEPS;
    h->m_valid = push;
    for (int64_t k = reps * GRAPH_STEPS; k < n; ++k) launch_step(h);
    return EVLBM_OK;
}

}  // namespace evlbm

// ================================================================ C ABI

extern "C" {

const char *evlbm_last_error(void) { return g_err; }

const char *evlbm_version(void) { return "evlbm gfx950 D2Q9/D3Q27 F64/F32/F16DEV/BF16DEV"; }

int evlbm_create(int lattice, int nx, int ny, int nz, int storage, void *stream, evlbm_t *out)
{
    if (!out) return fail(EVLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (lattice != EVLBM_D2Q9 && lattice != EVLBM_D3Q27) return fail(EVLBM_EINVAL, "unknown lattice %d", lattice);
    if (storage < EVLBM_F64 || storage > EVLBM_BF16DEV) return fail(EVLBM_EINVAL, "unknown storage %d", storage);
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(EVLBM_EINVAL, "lattice sizes must be positive");
    if (lattice == EVLBM_D2Q9 && nz != 1) return fail(EVLBM_EINVAL, "D2Q9 needs nz == 1");
    {
        // kernels address a cell of one direction or moment array by a 32-bit byte offset
        const double cells = (double)nx * ny * nz;
        const double elem = storage == EVLBM_F64 ? 8.0 : 4.0;  // widest per-cell element of any array
        if (cells * elem + DIR_PAD >= 4294967296.0)
            return fail(EVLBM_EINVAL, "lattice of %.0f cells: each per-direction array must stay below 4 GiB", cells);
    }
    evlbm_lattice *h = new evlbm_lattice();
    h->D = lattice;
    h->Q = lattice == EVLBM_D2Q9 ? 9 : 27;
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->N = (long)nx * ny * nz;
    // Consecutive direction arrays start DIR_PAD bytes past a multiple of the
    // array size: with a stride that is a power of two (or a multiple of
    // 4 KiB) the same cell of all 2Q arrays falls on the same HBM channels,
    // and the 2Q loads a wave issues per cell queue on them.
    h->ds = h->N + DIR_PAD / store_bytes(storage);
    h->storage = storage;
    h->stream = (hipStream_t)stream;
    hipGetDevice(&h->device);
    const size_t pop_bytes = (size_t)h->ds * 2 * h->Q * store_bytes(storage);
    const size_t m_bytes = (size_t)h->N * (h->D + 2) * real_bytes(storage);
    hipError_t e;
    for (int k = 0; k < 2; ++k) {
        e = hipMalloc(&h->buf[k], pop_bytes);
        if (e != hipSuccess) {
            evlbm_destroy(h);
            return fail(EVLBM_ENOMEM, "hipMalloc(%zu) for populations: %s", pop_bytes, hipGetErrorString(e));
        }
    }
    e = hipMalloc(&h->m, m_bytes);
    long shell_n = 0;
    dispatch<RunShellElems>(h, &shell_n);
    if (e == hipSuccess && shell_n > 0) {
        e = hipMalloc(&h->m_alt, m_bytes);
        if (e == hipSuccess) e = hipMalloc(&h->shell, (size_t)shell_n * real_bytes(storage));
    }
    if (e == hipSuccess) e = hipMalloc(&h->lap, (size_t)h->N * real_bytes(storage));
    if (e == hipSuccess && (storage == EVLBM_F16DEV || storage == EVLBM_BF16DEV))
        e = hipMalloc(&h->refst, (size_t)h->N * sizeof(float4));
    if (e != hipSuccess) {
        evlbm_destroy(h);
        return fail(EVLBM_ENOMEM, "hipMalloc for moment fields: %s", hipGetErrorString(e));
    }
    *out = h;
    return EVLBM_OK;
}

int evlbm_destroy(evlbm_t h)
{
    if (!h) return EVLBM_OK;
    for (int k = 0; k < 2; ++k)
        if (h->graph_exec_par[k]) hipGraphExecDestroy(h->graph_exec_par[k]);
    for (int k = 0; k < 2; ++k)
        if (h->buf[k] && h->own_buf) hipFree(h->buf[k]);
    if (h->m) hipFree(h->m);
    if (h->m_alt) hipFree(h->m_alt);
    if (h->shell) hipFree(h->shell);
    if (h->lap) hipFree(h->lap);
    if (h->wall_fh) (void)hipFree(h->wall_fh);
    if (h->wall_fld) (void)hipFree(h->wall_fld);
    if (h->refst) hipFree(h->refst);
    if (h->scratch) hipFree(h->scratch);
    delete h;
    return EVLBM_OK;
}

static void invalidate_graph(evlbm_t h)
{
    for (int k = 0; k < 2; ++k) {
        if (h->graph_exec_par[k]) hipGraphExecDestroy(h->graph_exec_par[k]);
        h->graph_exec_par[k] = nullptr;
    }
}

int evlbm_set_eos(evlbm_t h, double R, double a, double b, double kappa)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    if (!(R > 0) || !(a >= 0) || !(b >= 0) || !(kappa >= 0))
        return fail(EVLBM_EINVAL, "need R > 0 and a, b, kappa >= 0");
    h->R = R;
    h->a = a;
    h->b = b;
    h->kappa = kappa;
    invalidate_graph(h);
    return EVLBM_OK;
}

int evlbm_set_relaxation(evlbm_t h, double tau, double lambda)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    if (!(tau > 0) || !(lambda > 0)) return fail(EVLBM_EINVAL, "need tau > 0 and lambda > 0");
    if (tau > lambda) return fail(EVLBM_EINVAL, "need lambda >= tau (effective relaxation time >= 0)");
    h->tau = tau;
    h->lambda = lambda;
    invalidate_graph(h);
    return EVLBM_OK;
}

int evlbm_set_option(evlbm_t h, int key, double value)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    switch (key) {
    case EVLBM_OPT_SPHI:
        if (value != 1.0 && value != -1.0 && value != 0.0) return fail(EVLBM_EINVAL, "s_phi must be -1, 0 or +1");
        h->sphi = value;
        break;
    case EVLBM_OPT_CHECK_EVERY:
        if (value < 0) return fail(EVLBM_EINVAL, "check interval must be >= 0");
        h->check_every = (int64_t)value;
        break;
    case EVLBM_OPT_USE_GRAPH:
        h->use_graph = value != 0.0;
        break;
    case EVLBM_OPT_REREF_EVERY:
        if (value < 0) return fail(EVLBM_EINVAL, "re-reference period must be >= 0");
        h->reref_every = (int64_t)value;
        break;
    case EVLBM_OPT_PUSH_MOMENTS:
        h->push = value != 0.0;
        h->m_valid = false;
        break;
    case EVLBM_OPT_EOS:
        if (value != EVLBM_EOS_VDW && value != EVLBM_EOS_CS) return fail(EVLBM_EINVAL, "unknown pressure closure");
        h->eos = (int)value;
        break;
    case EVLBM_OPT_PRANDTL:
        if (!(value > 0) || !std::isfinite(value)) return fail(EVLBM_EINVAL, "the Prandtl number must be positive");
        h->prandtl = value;
        h->m_valid = false;
        break;
    default:
        return fail(EVLBM_EINVAL, "unknown option %d", key);
    }
    invalidate_graph(h);
    return EVLBM_OK;
}

int evlbm_init_fields(evlbm_t h, const void *rho, const void *u, const void *T, int where)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    if (!rho || !T) return fail(EVLBM_EINVAL, "rho and T are required");
    if (where != EVLBM_HOST_F64 && where != EVLBM_DEVICE_F32 && where != EVLBM_DEVICE_F64)
        return fail(EVLBM_EINVAL, "unknown location %d", where);
    const long N = h->N;
    const size_t need = sizeof(double) * N * (2 + h->D) + 64;
    int rc = ensure_scratch(h, need);
    if (rc) return rc;
    double *d_rho = (double *)h->scratch;
    double *d_T = d_rho + N;
    double *d_u = u ? d_T + N : nullptr;
    int *flag = (int *)(d_T + N + (long)h->D * N);
    hipError_t e = hipSuccess;
    if (where == EVLBM_HOST_F64) {
        const double *hr = (const double *)rho, *ht = (const double *)T;
        for (long c = 0; c < N; ++c) {
            if (!std::isfinite(hr[c]) || !std::isfinite(ht[c]))
                return fail(EVLBM_ENONFINITE, "non-finite initial field at cell %ld", c);
            double Z;
            if (!(hr[c] > 0) || !enskog_z64(h->eos, h->b, hr[c], &Z) || !(ht[c] > 0))
                return fail(EVLBM_ENONPHYS, "cell %ld: need rho > 0 inside the pressure closure's range, T > 0", c);
        }
        e = hipMemcpyAsync(d_rho, rho, sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(d_T, T, sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess && u)
            e = hipMemcpyAsync(d_u, u, sizeof(double) * N * h->D, hipMemcpyHostToDevice, h->stream);
    } else if (where == EVLBM_DEVICE_F64) {
        e = hipMemcpyAsync(d_rho, rho, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(d_T, T, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess && u)
            e = hipMemcpyAsync(d_u, u, sizeof(double) * N * h->D, hipMemcpyDeviceToDevice, h->stream);
    } else {
        const long nb = (N + 255) / 256;
        hipLaunchKernelGGL(k_f32_to_f64, dim3(nb), dim3(256), 0, h->stream, (const float *)rho, d_rho, N);
        hipLaunchKernelGGL(k_f32_to_f64, dim3(nb), dim3(256), 0, h->stream, (const float *)T, d_T, N);
        if (u)
            hipLaunchKernelGGL(k_f32_to_f64, dim3((N * h->D + 255) / 256), dim3(256), 0, h->stream, (const float *)u,
                               d_u, N * h->D);
    }
    if (e != hipSuccess) return hip_fail(e, "copying initial fields");
    if (where != EVLBM_HOST_F64) {
        int zero = 0, host = 0;
        e = hipMemcpyAsync(flag, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        hipLaunchKernelGGL(k_validate, dim3((N + 255) / 256), dim3(256), 0, h->stream, d_rho, d_T, N, h->eos, h->b,
                           flag);
        e = hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "validating initial fields");
        if (host & 2) return fail(EVLBM_ENONFINITE, "non-finite initial field");
        if (host & 1) return fail(EVLBM_ENONPHYS, "need rho > 0 inside the pressure closure's range, T > 0 everywhere");
    }
    h->cur = 0;
    if (h->refst) {
        if (h->D == 2)
            hipLaunchKernelGGL(k_ref_from_fields<2>, dim3((N + 255) / 256), dim3(256), 0, h->stream,
                               (const double *)d_rho, (const double *)d_T, N, h->R, h->eos, h->b, h->refst);
        else
            hipLaunchKernelGGL(k_ref_from_fields<3>, dim3((N + 255) / 256), dim3(256), 0, h->stream,
                               (const double *)d_rho, (const double *)d_T, N, h->R, h->eos, h->b, h->refst);
    }
    dispatch<RunInit>(h, (const double *)d_rho, (const double *)d_u, (const double *)d_T);
    rc = check_launch("k_init");
    if (rc) return rc;
    h->step = 0;
    h->initialized = true;
    h->m_valid = false;
    invalidate_graph(h);
    // the scratch buffer is reused by later calls: finish before returning
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return EVLBM_OK;
}

int evlbm_step(evlbm_t h, int64_t nsteps)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    if (!h->initialized) return fail(EVLBM_ESTATE, "lattice not initialised");
    if (nsteps < 0) return fail(EVLBM_EINVAL, "nsteps must be >= 0");
    int64_t done = 0;
    const int64_t reref = h->refst ? h->reref_every : 0;
    while (done < nsteps) {
        int64_t chunk = nsteps - done;
        if (h->check_every > 0) chunk = std::min<int64_t>(chunk, h->check_every - (h->step % h->check_every));
        if (reref > 0) chunk = std::min<int64_t>(chunk, reref - (h->step % reref));
        int rc = run_steps(h, chunk);
        if (rc) return rc;
        done += chunk;
        if (h->check_every > 0 && h->step % h->check_every == 0) {
            rc = scan_nonfinite(h);
            if (rc) return rc;
        }
        if (reref > 0 && h->step % reref == 0) {
            rc = rereference(h);
            if (rc) return rc;
        }
    }
    return check_launch("evlbm_step");
}

int evlbm_step_count(evlbm_t h, int64_t *out)
{
    if (!h || !out) return fail(EVLBM_EINVAL, "null argument");
    *out = h->step;
    return EVLBM_OK;
}

int evlbm_read_moments(evlbm_t h, void *rho, void *u, void *T, int where)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    if (!h->initialized) return fail(EVLBM_ESTATE, "lattice not initialised");
    if (where != EVLBM_HOST_F64 && where != EVLBM_DEVICE_F32 && where != EVLBM_DEVICE_F64)
        return fail(EVLBM_EINVAL, "unknown location %d", where);
    const long N = h->N;
    if (h->walls) {
        int rc = where == EVLBM_HOST_F64 ? ensure_scratch(h, sizeof(double) * N * (2 + h->D)) : EVLBM_OK;
        if (rc == EVLBM_OK) rc = wall_read_moments(h, rho, u, T, where, (double *)h->scratch);
        if (rc || where != EVLBM_HOST_F64) return rc;
        const double *d = (const double *)h->scratch;
        hipError_t e = hipSuccess;
        if (rho) e = hipMemcpyAsync(rho, d, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && T) e = hipMemcpyAsync(T, d + N, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && u)
            e = hipMemcpyAsync(u, d + 2 * N, sizeof(double) * N * h->D, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "copying moments to the host");
        return EVLBM_OK;
    }
    refresh_moments(h);
    dispatch<RunLap>(h);
    if (where == EVLBM_DEVICE_F32) {
        dispatch<RunReadoutF>(h, (float *)rho, (float *)u, (float *)T);
        return check_launch("readout");
    }
    if (where == EVLBM_DEVICE_F64) {
        dispatch<RunReadoutD>(h, (double *)rho, (double *)u, (double *)T);
        return check_launch("readout");
    }
    int rc = ensure_scratch(h, sizeof(double) * N * (2 + h->D));
    if (rc) return rc;
    double *d_rho = (double *)h->scratch, *d_T = d_rho + N, *d_u = d_T + N;
    dispatch<RunReadoutD>(h, d_rho, d_u, d_T);
    rc = check_launch("readout");
    if (rc) return rc;
    hipError_t e = hipSuccess;
    if (rho) e = hipMemcpyAsync(rho, d_rho, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && T) e = hipMemcpyAsync(T, d_T, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, d_u, sizeof(double) * N * h->D, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "copying moments to the host");
    return EVLBM_OK;
}

int evlbm_global_sums(evlbm_t h, double out[8])
{
    if (!h || !out) return fail(EVLBM_EINVAL, "null argument");
    if (!h->initialized) return fail(EVLBM_ESTATE, "lattice not initialised");
    const long nb = (h->N + 255) / 256;
    int rc = ensure_scratch(h, sizeof(double) * (nb * 9 + 16));
    if (rc) return rc;
    if (h->walls) {
        wall_sums(h, (double *)h->scratch);
    } else {
        refresh_moments(h);
        dispatch<RunLap>(h);
        dispatch<RunSums>(h, (double *)h->scratch, nb);
    }
    rc = check_launch("k_sums");
    if (rc) return rc;
    const int ops[8] = {0, 0, 0, 0, 0, 0, 1, 2};
    return finish_reduce(h, nb, 8, ops, out);
}

}  // extern "C"

// ------------------------------------------------- sums without allocation

// Device scratch of evlbm_global_sums_noalloc: the FP64 block partials of the
// reduction, 8 values for each block of 256 cells, for lattices of up to
// NOALLOC_MAX_CELLS cells (4 MiB).  One array per GPU, held until the process
// ends; host code never names it, only the per-device address that
// hipGetSymbolAddress returns for it (noalloc_scratch()).
static constexpr long NOALLOC_MAX_CELLS = 1L << 24;
static constexpr long NOALLOC_DOUBLES = 8 * (NOALLOC_MAX_CELLS / 256);
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mutex;
double *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// The address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
int noalloc_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(EVLBM_EINVAL, "device %d beyond the supported range", dev);
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_noalloc_ptr[dev] = (double *)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return EVLBM_OK;
}

}  // namespace

extern "C" {

int evlbm_global_sums_noalloc(evlbm_t h, double *out_dev)
{
    if (!h || !out_dev) return fail(EVLBM_EINVAL, "null argument");
    if (!h->initialized) return fail(EVLBM_ESTATE, "lattice not initialised");
    if (h->N > NOALLOC_MAX_CELLS)
        return fail(EVLBM_EINVAL, "lattice of %ld cells: the sums without allocation take at most %ld", h->N,
                    NOALLOC_MAX_CELLS);
    // the scratch belongs to the device the handle's stream runs on
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != h->device) return fail(EVLBM_EINVAL, "call with the lattice's device (%d) current", h->device);
    double *partial = nullptr;
    int rc = noalloc_scratch(&partial);
    if (rc) return rc;
    const long nb = (h->N + 255) / 256;
    // every block writes all of its 8 partials, so nothing needs clearing
    if (h->walls) {
        wall_sums(h, partial);
    } else {
        refresh_moments(h);
        dispatch<RunLap>(h);
        dispatch<RunSums>(h, partial, nb);
    }
    rc = check_launch("k_sums");
    if (rc) return rc;
    const int4 lo = make_int4(0, 0, 0, 0), hi = make_int4(0, 0, 1, 2);
    hipLaunchKernelGGL(k_reduce_final, dim3(8), dim3(256), 0, h->stream, (const double *)partial, nb, lo, hi, out_dev);
    return check_launch("reduce");
}

int evlbm_measure(evlbm_t h, int kind, const double *geom, double out[8])
{
    if (!h || !geom || !out) return fail(EVLBM_EINVAL, "null argument");
    if (!h->initialized) return fail(EVLBM_ESTATE, "lattice not initialised");
    if (kind != EVLBM_MEASURE_SLAB && kind != EVLBM_MEASURE_DROPLET) return fail(EVLBM_EINVAL, "unknown kind %d", kind);
    if (h->walls) return fail(EVLBM_EINVAL, "the region measurement is for periodic lattices (walls are set)");
    refresh_moments(h);
    dispatch<RunLap>(h);
    const long nb = (h->N + 255) / 256;
    int rc = ensure_scratch(h, sizeof(double) * (nb * 9 + 16));
    if (rc) return rc;
    double g[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < (kind == EVLBM_MEASURE_SLAB ? 6 : 5); ++k) g[k] = geom[k];
    dispatch<RunMeasure>(h, kind, (const double *)g, (double *)h->scratch, nb);
    rc = check_launch("k_measure");
    if (rc) return rc;
    const int ops[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double s[9];
    rc = finish_reduce(h, nb, 9, ops, s);
    if (rc) return rc;
    const double total = s[8];
    const double n_in = s[3], n_out = s[7];
    const double rin = n_in > 0 ? s[0] / n_in : NAN, rout = n_out > 0 ? s[4] / n_out : NAN;
    out[0] = rin;
    out[1] = rout;
    out[2] = n_in > 0 ? s[1] / n_in : NAN;
    out[3] = n_out > 0 ? s[5] / n_out : NAN;
    out[4] = n_in > 0 ? s[2] / n_in : NAN;
    out[5] = n_out > 0 ? s[6] / n_out : NAN;
    double Re = NAN;
    if (kind == EVLBM_MEASURE_DROPLET && n_in > 0 && n_out > 0) {
        const double vol = (total - (double)h->N * rout) / (rin - rout);
        Re = h->D == 2 || h->nz == 1 ? std::sqrt(vol / M_PI) : std::cbrt(3.0 * vol / (4.0 * M_PI));
    }
    out[6] = Re;
    out[7] = n_in;
    return EVLBM_OK;
}

int evlbm_get_populations(evlbm_t h, void *f, void *g, int where)
{
    if (!h || !f || !g) return fail(EVLBM_EINVAL, "null argument");
    if (where != EVLBM_HOST_F64 && where != EVLBM_DEVICE_F64) return fail(EVLBM_EINVAL, "populations are FP64");
    const size_t half = sizeof(double) * h->N * h->Q;
    int rc = ensure_scratch(h, 2 * half);
    if (rc) return rc;
    dispatch<RunDecode>(h, (double *)h->scratch);
    rc = check_launch("k_decode");
    if (rc) return rc;
    const hipMemcpyKind k = where == EVLBM_HOST_F64 ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    hipError_t e = hipMemcpyAsync(f, h->scratch, half, k, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(g, (char *)h->scratch + half, half, k, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "copying populations");
    return EVLBM_OK;
}

int evlbm_set_populations(evlbm_t h, const void *f, const void *g, int where)
{
    if (!h || !f || !g) return fail(EVLBM_EINVAL, "null argument");
    if (where != EVLBM_HOST_F64 && where != EVLBM_DEVICE_F64) return fail(EVLBM_EINVAL, "populations are FP64");
    const size_t half = sizeof(double) * h->N * h->Q;
    int rc = ensure_scratch(h, 2 * half);
    if (rc) return rc;
    const hipMemcpyKind k = where == EVLBM_HOST_F64 ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    hipError_t e = hipMemcpyAsync(h->scratch, f, half, k, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync((char *)h->scratch + half, g, half, k, h->stream);
    if (e != hipSuccess) return hip_fail(e, "copying populations");
    if (h->refst) dispatch<RunRefFromPops>(h, (const double *)h->scratch);
    dispatch<RunEncode>(h, (const double *)h->scratch);
    rc = check_launch("k_encode");
    if (rc) return rc;
    h->initialized = true;
    h->m_valid = false;
    invalidate_graph(h);
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return EVLBM_OK;
}

int evlbm_checkpoint_save(evlbm_t h, const char *path)
{
    if (!h || !path) return fail(EVLBM_EINVAL, "null argument");
    if (!h->initialized) return fail(EVLBM_ESTATE, "lattice not initialised");
    const size_t es = store_bytes(h->storage), row = (size_t)h->N * es;
    const size_t bytes = row * 2 * h->Q;
    // The one-pass step carries its moment field from step to step; saving it
    // makes a resumed run continue bit for bit (moments pulled again would
    // differ in rounding).
    const bool with_m = pushes(h);
    const size_t m_bytes = with_m ? (size_t)h->N * (h->D + 2) * real_bytes(h->storage) : 0;
    if (with_m) refresh_moments(h);
    std::vector<char> host(bytes), hm(m_bytes);
    hipError_t e = hipStreamSynchronize(h->stream);
    // dense [2Q][N] on disk: one row per direction array
    if (e == hipSuccess)
        e = hipMemcpy2D(host.data(), row, h->buf[h->cur], (size_t)h->ds * es, row, 2 * h->Q, hipMemcpyDeviceToHost);
    if (e == hipSuccess && with_m) e = hipMemcpy(hm.data(), h->m, m_bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copying populations");
    FILE *fp = fopen(path, "wb");
    if (!fp) return fail(EVLBM_EIO, "cannot open %s", path);
    char hdr[512];
    int n = snprintf(hdr, sizeof(hdr),
                     "{\"format\":\"evlbm-5\",\"lattice\":%d,\"nx\":%d,\"ny\":%d,\"nz\":%d,\"storage\":%d,"
                     "\"R\":%.17g,\"a\":%.17g,\"b\":%.17g,\"kappa\":%.17g,\"tau\":%.17g,\"lambda\":%.17g,"
                     "\"sphi\":%.17g,\"eos\":%d,\"Pr\":%.17g,\"walls\":%d,\"Tw\":%.17g,\"Uw\":%.17g,"
                     "\"step\":%lld,\"bytes\":%zu,\"moment_bytes\":%zu}\n",
                     h->D, h->nx, h->ny, h->nz, h->storage, h->R, h->a, h->b, h->kappa, h->tau, h->lambda, h->sphi,
                     h->eos, h->prandtl, h->walls ? 1 : 0, h->Tw, h->Uw, (long long)h->step, bytes, m_bytes);
    bool ok = fwrite(hdr, 1, n, fp) == (size_t)n && fwrite(host.data(), 1, bytes, fp) == bytes;
    if (ok && h->refst) {  // the 16-bit reference state of every cell
        std::vector<float4> r((size_t)h->N);
        e = hipMemcpy(r.data(), h->refst, sizeof(float4) * h->N, hipMemcpyDeviceToHost);
        ok = e == hipSuccess && fwrite(r.data(), sizeof(float4), h->N, fp) == (size_t)h->N;
    }
    if (ok && with_m) ok = fwrite(hm.data(), 1, m_bytes, fp) == m_bytes;
    ok = (fclose(fp) == 0) && ok;
    if (!ok) return fail(EVLBM_EIO, "writing %s failed", path);
    return EVLBM_OK;
}

int evlbm_checkpoint_load(evlbm_t h, const char *path)
{
    if (!h || !path) return fail(EVLBM_EINVAL, "null argument");
    FILE *fp = fopen(path, "rb");
    if (!fp) return fail(EVLBM_EIO, "cannot open %s", path);
    char hdr[1024];
    if (!fgets(hdr, sizeof(hdr), fp)) {
        fclose(fp);
        return fail(EVLBM_EIO, "empty checkpoint %s", path);
    }
    int D = 0, nx = 0, ny = 0, nz = 0, st = -1, eos = 0, walls = 0;
    double Tw = 0.0, Uw = 0.0, Pr = 1.0;
    long long step = 0;
    double R, a, b, kappa, tau, lam, sphi;
    size_t bytes = 0, m_bytes = 0;
    int got = sscanf(hdr,
                     "{\"format\":\"evlbm-5\",\"lattice\":%d,\"nx\":%d,\"ny\":%d,\"nz\":%d,\"storage\":%d,"
                     "\"R\":%lg,\"a\":%lg,\"b\":%lg,\"kappa\":%lg,\"tau\":%lg,\"lambda\":%lg,"
                     "\"sphi\":%lg,\"eos\":%d,\"Pr\":%lg,\"walls\":%d,\"Tw\":%lg,\"Uw\":%lg,\"step\":%lld,"
                     "\"bytes\":%zu,\"moment_bytes\":%zu}",
                     &D, &nx, &ny, &nz, &st, &R, &a, &b, &kappa, &tau, &lam, &sphi, &eos, &Pr, &walls, &Tw, &Uw, &step,
                     &bytes, &m_bytes);
    if (got != 20 || (eos != EVLBM_EOS_VDW && eos != EVLBM_EOS_CS) || !(Pr > 0)) {
        fclose(fp);
        return fail(EVLBM_EIO, "bad checkpoint header in %s", path);
    }
    if (D != h->D || nx != h->nx || ny != h->ny || nz != h->nz || st != h->storage) {
        fclose(fp);
        return fail(EVLBM_EINVAL, "checkpoint lattice/sizes/storage differ from the handle");
    }
    const size_t es = store_bytes(h->storage), row = (size_t)h->N * es;
    if (bytes != row * 2 * h->Q) {
        fclose(fp);
        return fail(EVLBM_EIO, "checkpoint %s holds %zu population bytes, expected %zu", path, bytes, row * 2 * h->Q);
    }
    std::vector<char> host(bytes);
    bool ok = fread(host.data(), 1, bytes, fp) == bytes;
    std::vector<float4> r;
    if (ok && h->refst) {
        r.resize((size_t)h->N);
        ok = fread(r.data(), sizeof(float4), h->N, fp) == (size_t)h->N;
    }
    const size_t m_need = (size_t)h->N * (h->D + 2) * real_bytes(h->storage);
    if (m_bytes != 0 && m_bytes != m_need) {
        fclose(fp);
        return fail(EVLBM_EIO, "checkpoint %s holds %zu moment bytes, expected %zu", path, m_bytes, m_need);
    }
    std::vector<char> hm(m_bytes);
    if (ok && m_bytes) ok = fread(hm.data(), 1, m_bytes, fp) == m_bytes;
    fclose(fp);
    if (!ok) return fail(EVLBM_EIO, "truncated checkpoint %s", path);
    if (h->refst) {
        hipError_t e2 = hipMemcpy(h->refst, r.data(), sizeof(float4) * h->N, hipMemcpyHostToDevice);
        if (e2 != hipSuccess) return hip_fail(e2, "copying the reference density");
    }
    h->R = R;
    h->a = a;
    h->b = b;
    h->kappa = kappa;
    h->tau = tau;
    h->lambda = lam;
    h->sphi = sphi;
    h->eos = eos;
    h->prandtl = Pr;
    if (walls) {
        const int rcw = evlbm_set_walls(h, 1, Tw, Uw);
        if (rcw) return rcw;
    } else {
        h->walls = false;
    }
    h->cur = 0;
    hipError_t e =
        hipMemcpy2D(h->buf[0], (size_t)h->ds * es, host.data(), row, row, 2 * h->Q, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "copying populations");
    // the saved moment field is used only by a handle taking the one-pass step
    const bool use_m = m_bytes != 0 && pushes(h);
    if (use_m) {
        e = hipMemcpy(h->m, hm.data(), m_bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "copying moments");
    }
    h->step = step;
    h->initialized = true;
    h->m_valid = use_m;
    invalidate_graph(h);
    return EVLBM_OK;
}

int evlbm_profile_step(evlbm_t h, int nsteps, double out[2])
{
    if (!h || !out || nsteps <= 0 || nsteps > 4096) return fail(EVLBM_EINVAL, "need 0 < nsteps <= 4096");
    if (!h->initialized) return fail(EVLBM_ESTATE, "lattice not initialised");
    if (h->walls) return fail(EVLBM_EINVAL, "kernel profiling is for periodic lattices (walls are set)");
    std::vector<hipEvent_t> ev((size_t)3 * nsteps, nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e == hipSuccess) {
        // two-pass step: [moments] [collision]; one-pass D3Q27: [collision]
        // [fix-up]; one-pass D2Q9: [nothing] [collision]
        const bool push = pushes(h);
        for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
            e = hipEventRecord(ev[3 * k], h->stream);
            if (!push && !fused(h)) {
                h->m_valid = false;
                refresh_moments(h);
            }
            launch_step(h, ev[3 * k + 1]);
            if (e == hipSuccess) e = hipEventRecord(ev[3 * k + 2], h->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    double tm = 0.0, tc = 0.0;
    const bool push = pushes(h);
    for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
        float a = 0.f, b = 0.f;
        e = hipEventElapsedTime(&a, ev[3 * k], ev[3 * k + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[3 * k + 1], ev[3 * k + 2]);
        tm += push ? b : a;
        tc += push ? a : b;
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(e, "profiling the step kernels");
    out[0] = tm / nsteps;
    out[1] = tc / nsteps;
    return EVLBM_OK;
}

int evlbm_population_bytes(evlbm_t h, size_t *bytes, long *stride)
{
    if (!h || !bytes) return fail(EVLBM_EINVAL, "null argument");
    *bytes = (size_t)h->ds * 2 * h->Q * store_bytes(h->storage);
    if (stride) *stride = h->ds;
    return EVLBM_OK;
}

int evlbm_attach_buffers(evlbm_t h, void *a, void *b, size_t bytes)
{
    if (!h || !a || !b) return fail(EVLBM_EINVAL, "null argument");
    size_t need = 0;
    evlbm_population_bytes(h, &need, nullptr);
    if (bytes < need) return fail(EVLBM_EINVAL, "population buffers of %zu bytes, need %zu", bytes, need);
    if (a == b) return fail(EVLBM_EINVAL, "the two population buffers must differ");
    if (((uintptr_t)a | (uintptr_t)b) % 256 != 0) return fail(EVLBM_EINVAL, "population buffers must be 256-byte aligned");
    const char *pa = (const char *)a, *pb = (const char *)b;
    if (pa < pb + need && pb < pa + need) return fail(EVLBM_EINVAL, "the two population buffers overlap");
    hipPointerAttribute_t at;
    for (void *ptr : {a, b}) {
        if (hipPointerGetAttributes(&at, ptr) != hipSuccess || at.type != hipMemoryTypeDevice || at.device != h->device)
            return fail(EVLBM_EINVAL, "population buffers must be device memory of the lattice's device");
    }
    (void)hipGetLastError();
    // the state moves with the buffers: copy both (the current one and the
    // other, which the next step overwrites) on the lattice's stream
    hipError_t e = hipMemcpyAsync(a, h->buf[0], need, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b, h->buf[1], need, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "attach population buffers");
    if (h->own_buf) {
        (void)hipFree(h->buf[0]);
        (void)hipFree(h->buf[1]);
    }
    h->buf[0] = a;
    h->buf[1] = b;
    h->own_buf = false;
    invalidate_graph(h);
    return EVLBM_OK;
}

int evlbm_synchronize(evlbm_t h)
{
    if (!h) return fail(EVLBM_EINVAL, "null handle");
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return EVLBM_OK;
}

namespace {

// Host thermodynamics of the bulk pressure P = rho RT Z(rho) - a rho^2 of a
// pressure closure (enskog_z64): P, dP/drho = RT (Z + rho Z') - 2 a rho and
// the chemical potential mu = RT [ln rho + f_ex/RT + Z - 1] - 2 a rho (up to a
// T-only constant; f_ex the hard-core excess free energy per particle):
//   van der Waals: Z + rho Z' = 1/(1 - b rho)^2, f_ex/RT = -ln(1 - b rho);
//   Carnahan-Starling (eta = b rho/4): Z + rho Z' = (1 + 4 eta + 4 eta^2 -
//     4 eta^3 + eta^4)/(1 - eta)^4, f_ex/RT + Z - 1 = (8 eta - 9 eta^2 +
//     3 eta^3)/(1 - eta)^3.
struct HostEos {
    int eos;
    double RT, a, b;
    double rmax() const { return eos == EVLBM_EOS_CS ? 4.0 / b : 1.0 / b; }
    double P(double r) const
    {
        double Z = 0.0;
        enskog_z64(eos, b, r, &Z);
        return r * RT * Z - a * r * r;
    }
    double dP(double r) const
    {
        if (eos == EVLBM_EOS_CS) {
            const double e = 0.25 * b * r, o = 1.0 - e;
            return RT * (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) / (o * o * o * o) - 2.0 * a * r;
        }
        return RT / ((1.0 - b * r) * (1.0 - b * r)) - 2.0 * a * r;
    }
    double mu(double r) const
    {
        if (eos == EVLBM_EOS_CS) {
            const double e = 0.25 * b * r, o = 1.0 - e;
            return RT * (std::log(r) + e * (8.0 + e * (-9.0 + 3.0 * e)) / (o * o * o)) - 2.0 * a * r;
        }
        return RT * std::log(r / (1.0 - b * r)) + RT / (1.0 - b * r) - 2.0 * a * r;
    }
};

// Critical point {rho_c, T_c, P_c}: closed form (van der Waals) or the
// bisection of s'(eta) = eta s''(eta) for s = 4 eta Z (Carnahan-Starling) with
// s' = 4 (1 + 4 eta + 4 eta^2 - 4 eta^3 + eta^4)/(1 - eta)^4 and
// s'' = 16 (2 + 5 eta - eta^2)/(1 - eta)^5, then R T_c = 32 a/(b s''(eta_c)).
void critical(int eos, double R, double a, double b, double out[3])
{
    if (eos == EVLBM_EOS_CS) {
        auto s1 = [](double e) {
            const double o = 1.0 - e;
            return 4.0 * (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) / (o * o * o * o);
        };
        auto s2 = [](double e) {
            const double o = 1.0 - e;
            return 16.0 * (2.0 + e * (5.0 - e)) / (o * o * o * o * o);
        };
        double lo = 0.01, hi = 0.5;  // s' - eta s'' changes sign once in between
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if ((s1(mid) - mid * s2(mid)) > 0.0) lo = mid;
            else hi = mid;
        }
        const double ec = 0.5 * (lo + hi), RTc = 32.0 * a / (b * s2(ec)), rc = 4.0 * ec / b;
        const HostEos th{eos, RTc, a, b};
        out[0] = rc;
        out[1] = RTc / R;
        out[2] = th.P(rc);
        return;
    }
    out[0] = 1.0 / (3.0 * b);
    out[1] = 8.0 * a / (27.0 * b * R);
    out[2] = a / (27.0 * b * b);
}

}  // namespace

int evlbm_eos_critical(int eos, double R, double a, double b, double out[3])
{
    if (!out || (eos != EVLBM_EOS_VDW && eos != EVLBM_EOS_CS)) return fail(EVLBM_EINVAL, "unknown pressure closure");
    if (!(R > 0) || !(a > 0) || !(b > 0)) return fail(EVLBM_EINVAL, "need R, a, b > 0");
    critical(eos, R, a, b, out);
    return EVLBM_OK;
}

int evlbm_eos_coexistence(int eos, double R, double a, double b, double T, double out[3])
{
    if (!out || (eos != EVLBM_EOS_VDW && eos != EVLBM_EOS_CS)) return fail(EVLBM_EINVAL, "unknown pressure closure");
    if (!(R > 0) || !(a > 0) || !(b > 0)) return fail(EVLBM_EINVAL, "need R, a, b > 0");
    double cp[3];
    critical(eos, R, a, b, cp);
    const double rc = cp[0], Tc = cp[1];
    if (!(T > 0) || !(T < Tc)) return fail(EVLBM_EINVAL, "T must lie in (0, T_c)");
    // Newton on P(rl) = P(rv), mu(rl) = mu(rv), continued in temperature from
    // just below T_c (where the mean-field critical law rho_c (1 +- 2 sqrt(1 -
    // T/Tc)) is a good start) down to T, each stage starting from the last;
    // damped so the iterates stay on their branches.
    const double eps0 = std::fmin(1e-3, 1.0 - T / Tc);
    const int stages = 48;
    double rl = 0.0, rv = 0.0;
    for (int k = 0; k <= stages; ++k) {
        // 1 - T_k/Tc from eps0 to 1 - T/Tc, geometrically
        const double eps = eps0 * std::pow((1.0 - T / Tc) / eps0, (double)k / stages);
        const HostEos th{eos, R * Tc * (1.0 - eps), a, b};
        const double rmax = th.rmax();
        if (k == 0) {
            rl = rc * (1.0 + 2.0 * std::sqrt(eps));
            rv = rc * (1.0 - 2.0 * std::sqrt(eps));
        }
        for (int it = 0; it < 100; ++it) {
            const double f1 = th.P(rl) - th.P(rv), f2 = th.mu(rl) - th.mu(rv);
            const double a11 = th.dP(rl), a12 = -th.dP(rv), a21 = th.dP(rl) / rl, a22 = -th.dP(rv) / rv;
            const double det = a11 * a22 - a12 * a21;
            const double drl = -(f1 * a22 - a12 * f2) / det, drv = -(a11 * f2 - a21 * f1) / det;
            double t = 1.0;
            while ((rl + t * drl >= rmax || rl + t * drl <= rc || rv + t * drv <= 0.0 || rv + t * drv >= rc) &&
                   t > 1e-6)
                t *= 0.5;
            rl += t * drl;
            rv += t * drv;
            if (std::fabs(drl) < 1e-15 * rl && std::fabs(drv) < 1e-15 * rv) break;
        }
    }
    const HostEos th{eos, R * T, a, b};
    out[0] = rl;
    out[1] = rv;
    out[2] = th.P(rl);
    if (!std::isfinite(rl) || !std::isfinite(rv) || !(rl > rc) || !(rv < rc))
        return fail(EVLBM_EINVAL, "coexistence iteration did not converge at T = %g", T);
    return EVLBM_OK;
}

}  // extern "C"


// ------------------------------------------------------------ copy probe

namespace evlbm {
// Plain streaming copy, 16 bytes per thread per iteration, grid-stride.
typedef float v4f __attribute__((ext_vector_type(4)));
// one 16-byte element per thread, non-temporal store: the streaming shape
// that reaches the highest copy rate on this part
__global__ void __launch_bounds__(256) k_copy_probe(const v4f *__restrict__ in, v4f *__restrict__ out, long n)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) __builtin_nontemporal_store(in[t], &out[t]);
}
}  // namespace evlbm

extern "C" int evlbm_copy_probe(double bytes, int reps, double *gbps_out)
{
    if (!gbps_out || !(bytes >= 1024) || reps <= 0) return fail(EVLBM_EINVAL, "need bytes >= 1024 and reps > 0");
    const long n = (long)(bytes / 2 / sizeof(v4f));  // half read, half written
    v4f *a = nullptr, *b = nullptr;
    hipError_t e = hipMalloc(&a, n * sizeof(v4f));
    if (e == hipSuccess) e = hipMalloc(&b, n * sizeof(v4f));
    if (e != hipSuccess) {
        if (a) (void)hipFree(a);
        return fail(EVLBM_ENOMEM, "copy probe allocation: %s", hipGetErrorString(e));
    }
    (void)hipMemset(a, 0, n * sizeof(v4f));
    const long blocks = (n + 255) / 256;
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    hipLaunchKernelGGL(k_copy_probe, dim3(blocks), dim3(256), 0, nullptr, a, b, n);
    (void)hipEventRecord(t0, nullptr);
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_copy_probe, dim3(blocks), dim3(256), 0, nullptr, a, b, n);
    (void)hipEventRecord(t1, nullptr);
    e = hipEventSynchronize(t1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(a);
    (void)hipFree(b);
    if (e != hipSuccess) return hip_fail(e, "copy probe");
    *gbps_out = 2.0 * n * sizeof(v4f) * reps / (ms * 1e-3) / 1e9;
    return EVLBM_OK;
}
