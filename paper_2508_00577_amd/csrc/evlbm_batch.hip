// Batched D2Q9 domains of uneven sizes (a temperature or size sweep) advanced
// together: one population arena, a device table of domains and a list of
// BX x BY tiles covering all of them; each step is one persistent launch of
// the stencil + collision kernel, whose workgroups stride over the whole tile
// list and sum each tile's halo moments from the pulled populations (the
// moment kernel runs only for readouts).  Step chunks are replayed from
// captured hipGraphs.  The tile shape is chosen by an autotuner among the
// compiled shapes.  Every cell runs the same device code as a single lattice,
// so a domain of the batch evolves bit for bit as the same domain alone with
// the same tile shape.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "evlbm_internal.hpp"
#include "evlbm_params.hpp"
#include "lbm_kernels.hpp"

using namespace evlbm;

namespace evlbm {

struct DomainRec {
    int nx, ny;
    long N;
    long pop_off;   // elements into the population arena (2Q N per domain)
    long m_off;     // elements into the moment arena ((D+2) N per domain)
    long cell_off;  // cells before this domain (reference-density arena)
};

// Compiled tile shapes: (BX, BY); variant 1 is a single lattice's D2Q9 tile
static constexpr int NVARIANT = 4;
static constexpr int VBX[NVARIANT] = {64, 64, 128, 64};
static constexpr int VBY[NVARIANT] = {4, 16, 2, 8};

template <typename R>
__device__ inline StepParams<R> domain_params(const StepParams<R> &p, const DomainRec &d)
{
    StepParams<R> q = p;
    q.nx = d.nx;
    q.ny = d.ny;
    q.nz = 1;
    q.N = d.N;
    q.ds = d.N;  // a domain's direction arrays are dense in the arena
    q.refst = p.refst ? p.refst + d.cell_off : nullptr;
    return q;
}

template <int S, int BX, int BY>
__global__ void __launch_bounds__(BX *BY)
    k_batch_moments(const StoreT<S> *__restrict__ pop, RealT<S> *__restrict__ m, const DomainRec *__restrict__ dom,
                    const int4 *__restrict__ tiles, int ntiles, StepParams<RealT<S>> p)
{
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const DomainRec d = dom[tl.x];
        const StepParams<RealT<S>> q = domain_params(p, d);
        const int x = tl.y + threadIdx.x, y = tl.z + threadIdx.y;
        if (x < d.nx && y < d.ny) moments_at<2, S>(pop + d.pop_off, m + d.m_off, q, x, y, 0);
    }
}

template <int S, int BX, int BY, bool VPR = false>
__global__ void __launch_bounds__(BX *BY)
    k_batch_collide(const StoreT<S> *__restrict__ src, StoreT<S> *__restrict__ dst, const RealT<S> *__restrict__ m,
                    const DomainRec *__restrict__ dom, const int4 *__restrict__ tiles, int ntiles,
                    StepParams<RealT<S>> p)
{
    // rounds of gridDim.x consecutive tiles; within a full round each XCD
    // takes a contiguous run of the list (xcd_tile), neighbouring tiles of
    // one domain, so their shared halo lines meet in one L2
    for (int r = 0; r < ntiles; r += gridDim.x) {
        const int t = r + (ntiles - r >= (int)gridDim.x ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x);
        if (t >= ntiles) break;
        const int4 tl = tiles[t];
        const DomainRec d = dom[tl.x];
        const StepParams<RealT<S>> q = domain_params(p, d);
        collide_block<2, S, BX, BY, 1, true, VPR>(src + d.pop_off, dst + d.pop_off, m + d.m_off, q, tl.y, tl.z, 0);
        __syncthreads();  // the next tile reuses the LDS staging buffers
    }
}

}  // namespace evlbm

struct evlbm_batch {
    int n = 0, storage = EVLBM_F32, Q = 9, D = 2;
    hipStream_t stream = nullptr;
    std::vector<DomainRec> doms;
    long cells = 0;
    void *buf[2] = {nullptr, nullptr};
    void *m = nullptr;
    void *lap = nullptr;
    float4 *refst = nullptr;  // 16-bit storage: reference state per cell of every domain
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    DomainRec *d_dom = nullptr;
    int4 *d_tiles[NVARIANT] = {nullptr, nullptr, nullptr, nullptr};
    int ntiles[NVARIANT] = {0, 0, 0, 0};
    int grid[NVARIANT][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // persistent grid: moments, collide (Pr = 1, Pr != 1)
    int variant = 0;
    double R = 1.0, a = 0.0, b = 0.0, kappa = 0.0, tau = 1.0, lambda = 1.0, sphi = -1.0;
    int eos = EVLBM_EOS_VDW;
    double prandtl = 1.0;
    int cur = 0;
    int64_t step = 0;
    int64_t reref_every = 100;  // 16-bit storage: re-reference period in steps (as a lattice's default)
    bool m_valid = false;
    std::vector<char> initialized;
    hipGraphExec_t graph_exec_par[2] = {nullptr, nullptr};
};

namespace {

size_t sbytes(int st) { return st == EVLBM_F64 ? 8 : st == EVLBM_F32 ? 4 : 2; }
size_t rbytes(int st) { return st == EVLBM_F64 ? 8 : 4; }

void drop_graphs(evlbm_batch *b)
{
    for (int k = 0; k < 2; ++k) {
        if (b->graph_exec_par[k]) (void)hipGraphExecDestroy(b->graph_exec_par[k]);
        b->graph_exec_par[k] = nullptr;
    }
}

int scratch(evlbm_batch *b, size_t bytes)
{
    if (b->scratch_bytes >= bytes) return EVLBM_OK;
    if (b->scratch) (void)hipFree(b->scratch);
    b->scratch = nullptr;
    b->scratch_bytes = 0;
    hipError_t e = hipMalloc(&b->scratch, bytes);
    if (e != hipSuccess) return fail(EVLBM_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    b->scratch_bytes = bytes;
    return EVLBM_OK;
}

template <typename R>
StepParams<R> bparams(const evlbm_batch *b)
{
    StepParams<R> p = model_params<R>(b->eos, b->R, b->a, b->b, b->kappa, b->tau, b->lambda, b->sphi, b->prandtl);
    p.refst = b->refst;
    return p;
}

template <typename R>
StepParams<R> dparams(const evlbm_batch *b, int k)
{
    StepParams<R> p = bparams<R>(b);
    const DomainRec &d = b->doms[k];
    p.nx = d.nx;
    p.ny = d.ny;
    p.nz = 1;
    p.N = d.N;
    p.ds = d.N;
    p.refst = b->refst ? b->refst + d.cell_off : nullptr;
    return p;
}

template <int S, int V>
struct BOps {
    using T = StoreT<S>;
    using R = RealT<S>;
    static constexpr int BX = VBX[V], BY = VBY[V];
    static void moments(evlbm_batch *b, const void *pop)
    {
        hipLaunchKernelGGL((k_batch_moments<S, BX, BY>), dim3(b->grid[V][0]), dim3(BX, BY), 0, b->stream,
                           (const T *)pop, (R *)b->m, b->d_dom, b->d_tiles[V], b->ntiles[V], bparams<R>(b));
    }
    static void collide(evlbm_batch *b, const void *src, void *dst)
    {
        // Prandtl number != 1: the collision with the quasi-equilibrium term
        if (b->prandtl != 1.0)
            hipLaunchKernelGGL((k_batch_collide<S, BX, BY, true>), dim3(b->grid[V][2]), dim3(BX, BY), 0, b->stream,
                               (const T *)src, (T *)dst, (const R *)b->m, b->d_dom, b->d_tiles[V], b->ntiles[V],
                               bparams<R>(b));
        else
            hipLaunchKernelGGL((k_batch_collide<S, BX, BY>), dim3(b->grid[V][1]), dim3(BX, BY), 0, b->stream,
                               (const T *)src, (T *)dst, (const R *)b->m, b->d_dom, b->d_tiles[V], b->ntiles[V],
                               bparams<R>(b));
    }
    static void occupancy(evlbm_batch *b, int cus)
    {
        int nm = 0, nc = 0, nv = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nm, k_batch_moments<S, BX, BY>, BX * BY, 0);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nc, k_batch_collide<S, BX, BY>, BX * BY, 0);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nv, k_batch_collide<S, BX, BY, true>, BX * BY, 0);
        b->grid[V][0] = std::max(1, std::min(b->ntiles[V], cus * std::max(nm, 1)));
        b->grid[V][1] = std::max(1, std::min(b->ntiles[V], cus * std::max(nc, 1)));
        b->grid[V][2] = std::max(1, std::min(b->ntiles[V], cus * std::max(nv, 1)));
    }
};

template <int S>
struct BDispatchS {
    static void moments(evlbm_batch *b, const void *pop)
    {
        switch (b->variant) {
        case 0: BOps<S, 0>::moments(b, pop); break;
        case 1: BOps<S, 1>::moments(b, pop); break;
        case 2: BOps<S, 2>::moments(b, pop); break;
        default: BOps<S, 3>::moments(b, pop); break;
        }
    }
    static void collide(evlbm_batch *b, const void *src, void *dst)
    {
        switch (b->variant) {
        case 0: BOps<S, 0>::collide(b, src, dst); break;
        case 1: BOps<S, 1>::collide(b, src, dst); break;
        case 2: BOps<S, 2>::collide(b, src, dst); break;
        default: BOps<S, 3>::collide(b, src, dst); break;
        }
    }
    static void occupancy(evlbm_batch *b, int cus)
    {
        BOps<S, 0>::occupancy(b, cus);
        BOps<S, 1>::occupancy(b, cus);
        BOps<S, 2>::occupancy(b, cus);
        BOps<S, 3>::occupancy(b, cus);
    }
    // 16-bit storage: re-reference domain k in place (as on a lattice)
    static void rereference(evlbm_batch *b, int k)
    {
        if constexpr (S == EVLBM_F16DEV || S == EVLBM_BF16DEV) {
            const DomainRec &d = b->doms[k];
            hipLaunchKernelGGL((k_rereference<2, S>), dim3((d.N + 255) / 256), dim3(256), 0, b->stream,
                               (StoreT<S> *)b->buf[b->cur] + d.pop_off, b->refst + d.cell_off,
                               dparams<RealT<S>>(b, k));
        }
    }
    // single-domain helpers (initialisation, readout, population I/O)
    static void init(evlbm_batch *b, int k, const double *rho, const double *u, const double *T0)
    {
        const DomainRec &d = b->doms[k];
        hipLaunchKernelGGL((k_init<2, S>), dim3((d.N + 255) / 256), dim3(256), 0, b->stream, rho, u, T0,
                           (StoreT<S> *)b->buf[b->cur] + d.pop_off, dparams<RealT<S>>(b, k));
    }
    static void decode(evlbm_batch *b, int k, double *out)
    {
        const DomainRec &d = b->doms[k];
        const long n = d.N * 18;
        hipLaunchKernelGGL((k_decode<2, S>), dim3((n + 255) / 256), dim3(256), 0, b->stream,
                           (const StoreT<S> *)b->buf[b->cur] + d.pop_off, out, d.N, 18, dparams<RealT<S>>(b, k));
    }
    static void readout(evlbm_batch *b, int k, double *rho, double *u, double *T0)
    {
        using R = RealT<S>;
        const DomainRec &d = b->doms[k];
        const int bx = d.nx >= 256 ? 256 : ((d.nx + 63) / 64) * 64;
        dim3 grid((d.nx + bx - 1) / bx, d.ny, 1);
        const R *m = (const R *)b->m + d.m_off;
        R *lap = (R *)b->lap + d.cell_off;
        hipLaunchKernelGGL((k_lap_field<2, R>), grid, dim3(bx), 0, b->stream, m, lap, d.nx, d.ny, 1);
        hipLaunchKernelGGL((k_readout<2, R, double>), grid, dim3(bx), 0, b->stream, m, (const R *)lap, rho, u, T0,
                           d.nx, d.ny, 1, (R)b->a, (R)b->kappa, (R)b->R);
    }
};

#define BATCH_DISPATCH(call)                                    \
    switch (b->storage) {                                       \
    case EVLBM_F64: BDispatchS<EVLBM_F64>::call; break;         \
    case EVLBM_F32: BDispatchS<EVLBM_F32>::call; break;         \
    case EVLBM_F16DEV: BDispatchS<EVLBM_F16DEV>::call; break;   \
    default: BDispatchS<EVLBM_BF16DEV>::call; break;            \
    }

// One step: the collision sums each tile's halo moments from the pulled
// populations (the one-pass D2Q9 step), so no moment pass runs.
void bstep(evlbm_batch *b)
{
    BATCH_DISPATCH(collide(b, b->buf[b->cur], b->buf[1 - b->cur]));
    b->cur = 1 - b->cur;
    b->m_valid = false;
    b->step++;
}

constexpr int BGRAPH_STEPS = 32;

int brun(evlbm_batch *b, int64_t n, bool use_graph)
{
    if (!use_graph || b->stream == nullptr || n < BGRAPH_STEPS) {
        for (int64_t k = 0; k < n; ++k) bstep(b);
        return EVLBM_OK;
    }
    const int par = b->cur;
    if (!b->graph_exec_par[par]) {
        const int cur0 = b->cur;
        const int64_t step0 = b->step;
        b->m_valid = false;
        hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        for (int k = 0; k < BGRAPH_STEPS; ++k) bstep(b);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->stream, &g);
        b->cur = cur0;
        b->step = step0;
        b->m_valid = false;
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        b->graph_exec_par[par] = ex;
    }
    const int64_t reps = n / BGRAPH_STEPS;
    for (int64_t r = 0; r < reps; ++r) {
        hipError_t e = hipGraphLaunch(b->graph_exec_par[par], b->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    b->step += reps * BGRAPH_STEPS;
    b->m_valid = false;
    for (int64_t k = reps * BGRAPH_STEPS; k < n; ++k) bstep(b);
    return EVLBM_OK;
}

}  // namespace

extern "C" {

int evlbm_batch_destroy(evlbm_batch_t b)
{
    if (!b) return EVLBM_OK;
    drop_graphs(b);
    for (int k = 0; k < 2; ++k)
        if (b->buf[k]) (void)hipFree(b->buf[k]);
    if (b->m) (void)hipFree(b->m);
    if (b->lap) (void)hipFree(b->lap);
    if (b->refst) (void)hipFree(b->refst);
    if (b->scratch) (void)hipFree(b->scratch);
    if (b->d_dom) (void)hipFree(b->d_dom);
    for (int v = 0; v < NVARIANT; ++v)
        if (b->d_tiles[v]) (void)hipFree(b->d_tiles[v]);
    delete b;
    return EVLBM_OK;
}

int evlbm_batch_create(int n, const evlbm_domain_desc *d, int storage, void *stream, evlbm_batch_t *out)
{
    if (!out || !d || n <= 0) return fail(EVLBM_EINVAL, "need n > 0 domains");
    *out = nullptr;
    if (storage < EVLBM_F64 || storage > EVLBM_BF16DEV) return fail(EVLBM_EINVAL, "unknown storage %d", storage);
    for (int k = 0; k < n; ++k)
        if (d[k].nx <= 0 || d[k].ny <= 0) return fail(EVLBM_EINVAL, "domain %d: sizes must be positive", k);
    evlbm_batch *b = new evlbm_batch();
    b->n = n;
    b->storage = storage;
    b->stream = (hipStream_t)stream;
    long pop = 0, mo = 0, cells = 0;
    for (int k = 0; k < n; ++k) {
        DomainRec r;
        r.nx = d[k].nx;
        r.ny = d[k].ny;
        r.N = (long)r.nx * r.ny;
        r.pop_off = pop;
        r.m_off = mo;
        r.cell_off = cells;
        pop += 18 * r.N;
        mo += 4 * r.N;
        cells += r.N;
        b->doms.push_back(r);
    }
    b->cells = cells;
    b->initialized.assign(n, 0);
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMalloc(&b->buf[k], (size_t)pop * sbytes(storage));
    if (e == hipSuccess) e = hipMalloc(&b->m, (size_t)mo * rbytes(storage));
    if (e == hipSuccess) e = hipMalloc(&b->lap, (size_t)cells * rbytes(storage));
    if (e == hipSuccess && (storage == EVLBM_F16DEV || storage == EVLBM_BF16DEV))
        e = hipMalloc(&b->refst, (size_t)cells * sizeof(float4));
    if (e == hipSuccess) e = hipMalloc(&b->d_dom, sizeof(DomainRec) * n);
    if (e == hipSuccess) e = hipMemcpy(b->d_dom, b->doms.data(), sizeof(DomainRec) * n, hipMemcpyHostToDevice);
    // tile lists per compiled shape, domain by domain, row-major tiles
    for (int v = 0; v < NVARIANT && e == hipSuccess; ++v) {
        std::vector<int4> tl;
        for (int k = 0; k < n; ++k)
            for (int y0 = 0; y0 < b->doms[k].ny; y0 += VBY[v])
                for (int x0 = 0; x0 < b->doms[k].nx; x0 += VBX[v]) tl.push_back(make_int4(k, x0, y0, 0));
        b->ntiles[v] = (int)tl.size();
        e = hipMalloc(&b->d_tiles[v], sizeof(int4) * tl.size());
        if (e == hipSuccess) e = hipMemcpy(b->d_tiles[v], tl.data(), sizeof(int4) * tl.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        evlbm_batch_destroy(b);
        return fail(EVLBM_ENOMEM, "batch allocation: %s", hipGetErrorString(e));
    }
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    BATCH_DISPATCH(occupancy(b, cus));
    *out = b;
    return EVLBM_OK;
}

int evlbm_batch_set_params(evlbm_batch_t b, double R, double a, double bb, double kappa, double tau, double lambda,
                           double sphi)
{
    if (!b) return fail(EVLBM_EINVAL, "null batch");
    if (!(R > 0) || !(a >= 0) || !(bb >= 0) || !(kappa >= 0)) return fail(EVLBM_EINVAL, "need R > 0, a, b, kappa >= 0");
    if (!(tau > 0) || !(lambda >= tau)) return fail(EVLBM_EINVAL, "need 0 < tau <= lambda");
    b->R = R;
    b->a = a;
    b->b = bb;
    b->kappa = kappa;
    b->tau = tau;
    b->lambda = lambda;
    b->sphi = sphi;
    drop_graphs(b);
    return EVLBM_OK;
}

int evlbm_batch_set_option(evlbm_batch_t b, int key, double value)
{
    if (!b) return fail(EVLBM_EINVAL, "null batch");
    switch (key) {
    case EVLBM_OPT_SPHI:
        if (value != 1.0 && value != -1.0 && value != 0.0) return fail(EVLBM_EINVAL, "s_phi must be -1, 0 or +1");
        b->sphi = value;
        break;
    case EVLBM_OPT_REREF_EVERY:
        if (value < 0) return fail(EVLBM_EINVAL, "re-reference period must be >= 0");
        b->reref_every = (int64_t)value;
        break;
    case EVLBM_OPT_EOS:
        if (value != EVLBM_EOS_VDW && value != EVLBM_EOS_CS) return fail(EVLBM_EINVAL, "unknown pressure closure");
        b->eos = (int)value;
        break;
    case EVLBM_OPT_PRANDTL:
        if (!(value > 0) || !std::isfinite(value)) return fail(EVLBM_EINVAL, "the Prandtl number must be positive");
        b->prandtl = value;
        break;
    default:
        return fail(EVLBM_EINVAL, "option %d is not a batch option", key);
    }
    drop_graphs(b);
    return EVLBM_OK;
}

int evlbm_batch_init_domain(evlbm_batch_t b, int k, const double *rho, const double *u, const double *T)
{
    if (!b || k < 0 || k >= b->n || !rho || !T) return fail(EVLBM_EINVAL, "bad domain index or null field");
    const DomainRec &d = b->doms[k];
    for (long c = 0; c < d.N; ++c) {
        if (!std::isfinite(rho[c]) || !std::isfinite(T[c])) return fail(EVLBM_ENONFINITE, "non-finite field");
        double Z;
        if (!(rho[c] > 0) || !enskog_z64(b->eos, b->b, rho[c], &Z) || !(T[c] > 0))
            return fail(EVLBM_ENONPHYS, "domain %d cell %ld: need rho > 0 inside the pressure closure's range, T > 0",
                        k, c);
    }
    int rc = scratch(b, sizeof(double) * d.N * 4);
    if (rc) return rc;
    double *dr = (double *)b->scratch, *dt = dr + d.N, *du = u ? dt + d.N : nullptr;
    hipError_t e = hipMemcpyAsync(dr, rho, sizeof(double) * d.N, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, T, sizeof(double) * d.N, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(du, u, sizeof(double) * 2 * d.N, hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return hip_fail(e, "copying initial fields");
    if (b->refst)
        hipLaunchKernelGGL(k_ref_from_fields<2>, dim3((d.N + 255) / 256), dim3(256), 0, b->stream, (const double *)dr,
                           (const double *)dt, d.N, b->R, b->eos, b->b, b->refst + d.cell_off);
    BATCH_DISPATCH(init(b, k, dr, du, dt));
    e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "initialising a domain");
    b->initialized[k] = 1;
    b->m_valid = false;
    return EVLBM_OK;
}

int evlbm_batch_step(evlbm_batch_t b, int64_t nsteps)
{
    if (!b) return fail(EVLBM_EINVAL, "null batch");
    for (int k = 0; k < b->n; ++k)
        if (!b->initialized[k]) return fail(EVLBM_ESTATE, "domain %d not initialised", k);
    if (nsteps < 0) return fail(EVLBM_EINVAL, "nsteps must be >= 0");
    const bool dev16 = b->storage == EVLBM_F16DEV || b->storage == EVLBM_BF16DEV;
    const int64_t reref = dev16 ? b->reref_every : 0;
    int64_t done = 0;
    while (done < nsteps) {
        int64_t chunk = nsteps - done;
        if (reref > 0) chunk = std::min<int64_t>(chunk, reref - (b->step % reref));
        int rc = brun(b, chunk, true);
        if (rc) return rc;
        done += chunk;
        if (reref > 0 && b->step % reref == 0) {
            for (int k = 0; k < b->n; ++k) BATCH_DISPATCH(rereference(b, k));
            b->m_valid = false;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batch step");
    return EVLBM_OK;
}

int evlbm_batch_read(evlbm_batch_t b, int k, double *rho, double *u, double *T)
{
    if (!b || k < 0 || k >= b->n) return fail(EVLBM_EINVAL, "bad domain index");
    const DomainRec &d = b->doms[k];
    if (!b->m_valid) {
        BATCH_DISPATCH(moments(b, b->buf[b->cur]));
        b->m_valid = true;
    }
    int rc = scratch(b, sizeof(double) * d.N * 4);
    if (rc) return rc;
    double *dr = (double *)b->scratch, *dt = dr + d.N, *du = dt + d.N;
    BATCH_DISPATCH(readout(b, k, dr, du, dt));
    hipError_t e = hipSuccess;
    if (rho) e = hipMemcpyAsync(rho, dr, sizeof(double) * d.N, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess && T) e = hipMemcpyAsync(T, dt, sizeof(double) * d.N, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, du, sizeof(double) * 2 * d.N, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch readout");
    return EVLBM_OK;
}

int evlbm_batch_get_populations(evlbm_batch_t b, int k, double *f, double *g)
{
    if (!b || k < 0 || k >= b->n || !f || !g) return fail(EVLBM_EINVAL, "bad argument");
    const DomainRec &d = b->doms[k];
    int rc = scratch(b, sizeof(double) * d.N * 18);
    if (rc) return rc;
    BATCH_DISPATCH(decode(b, k, (double *)b->scratch));
    hipError_t e = hipMemcpyAsync(f, b->scratch, sizeof(double) * 9 * d.N, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g, (double *)b->scratch + 9 * d.N, sizeof(double) * 9 * d.N, hipMemcpyDeviceToHost,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch populations");
    return EVLBM_OK;
}

int evlbm_batch_set_tile(evlbm_batch_t b, int variant)
{
    if (!b || variant < 0 || variant >= NVARIANT) return fail(EVLBM_EINVAL, "tile variant must be 0..%d", NVARIANT - 1);
    if (variant != b->variant) drop_graphs(b);
    b->variant = variant;
    return EVLBM_OK;
}

int evlbm_batch_info(evlbm_batch_t b, int64_t *cells, int *ntiles, int *variant, int *tile_x, int *tile_y)
{
    if (!b) return fail(EVLBM_EINVAL, "null batch");
    if (cells) *cells = b->cells;
    if (ntiles) *ntiles = b->ntiles[b->variant];
    if (variant) *variant = b->variant;
    if (tile_x) *tile_x = VBX[b->variant];
    if (tile_y) *tile_y = VBY[b->variant];
    return EVLBM_OK;
}

int evlbm_batch_autotune(evlbm_batch_t b, int steps, int *best, double *ms_per_step)
{
    if (!b || steps <= 0 || steps > 1000) return fail(EVLBM_EINVAL, "need 0 < steps <= 1000");
    for (int k = 0; k < b->n; ++k)
        if (!b->initialized[k]) return fail(EVLBM_ESTATE, "domain %d not initialised", k);
    // time every compiled tile shape on the real batch, then restore the state
    const size_t bytes = (size_t)b->cells * 18 * sbytes(b->storage);
    void *backup = nullptr;
    hipError_t e = hipMalloc(&backup, bytes);
    if (e != hipSuccess) return fail(EVLBM_ENOMEM, "autotune backup: %s", hipGetErrorString(e));
    e = hipMemcpyAsync(backup, b->buf[b->cur], bytes, hipMemcpyDeviceToDevice, b->stream);
    const int cur0 = b->cur;
    const int64_t step0 = b->step;
    const int v0 = b->variant;
    double best_ms = 1e300;
    int best_v = v0;
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    for (int v = 0; v < NVARIANT && e == hipSuccess; ++v) {
        b->variant = v;
        bstep(b);  // warm-up
        (void)hipEventRecord(t0, b->stream);
        for (int s = 0; s < steps; ++s) bstep(b);
        (void)hipEventRecord(t1, b->stream);
        e = hipEventSynchronize(t1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        const double per = ms / steps;
        if (ms_per_step) ms_per_step[v] = per;
        if (per < best_ms) {
            best_ms = per;
            best_v = v;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    b->cur = cur0;
    if (e == hipSuccess) e = hipMemcpyAsync(b->buf[cur0], backup, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(backup);
    b->step = step0;
    b->m_valid = false;
    b->variant = best_v;
    drop_graphs(b);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (best) *best = best_v;
    return EVLBM_OK;
}

}  // extern "C"
