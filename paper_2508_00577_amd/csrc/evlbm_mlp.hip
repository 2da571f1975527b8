// Warm-start network for droplet initialisation: inputs (T/Tc, R, r/R), three
// hidden layers of 64 tanh units, one linear output (density over the
// critical density).  FP32 parameters, trained on the GPU with these kernels:
// each wavefront takes 16 samples; the 64 x 64 layers run on the matrix cores
// (v_mfma_f32_16x16x4_f32) forward and backward, the 3 -> 64 and 64 -> 1
// layers on the vector ALUs; per-wave partial gradients are summed in a fixed
// order by the Adam kernel, so training is deterministic.
//
// Flat parameter layout (8641 floats): W1[64][3], b1[64], W2[64][64], b2[64],
// W3[64][64], b3[64], W4[64], b4.  Inputs are normalised as
// x1 = (T/Tc - 0.8)/0.15, x2 = (R - 47.5)/32.5, x3 = r/R - 1.
#include <cmath>
#include <vector>

#include "evlbm_internal.hpp"

using namespace evlbm;

namespace evlbm {

constexpr int H = 64;
constexpr int NPARAM = H * 3 + H + H * H + H + H * H + H + H + 1;  // 8641
constexpr int OW1 = 0, OB1 = OW1 + H * 3, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H * H,
              OW4 = OB3 + H, OB4 = OW4 + H;
constexpr int ROWS = 16;  // samples per wavefront

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline floatx4 mfma4(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Operand layout of v_mfma_f32_16x16x4_f32 (one 16 x 16 x 4 block), lane l:
//   A[i][k] with i = l % 16, k = l / 16;  B[k][j] with k = l / 16, j = l % 16;
//   D[i][j] in four registers r with i = 4 (l / 16) + r, j = l % 16.

// C[16 x 64] += A[16 x 64] * B[64 x 64]; A row-major in LDS (stride 64),
// B(k, j) = Bp[k * bk + j * bj]; acc[jt] holds columns 16 jt .. 16 jt + 15.
__device__ inline void wave_gemm_16x64(const float *A, const float *Bp, int bk, int bj, floatx4 acc[4])
{
    const int l = threadIdx.x & 63, i = l & 15, kk = l >> 4;
#pragma unroll 4
    for (int s = 0; s < H / 4; ++s) {
        const float a = A[i * H + 4 * s + kk];
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) acc[jt] = mfma4(a, Bp[(4 * s + kk) * bk + (16 * jt + i) * bj], acc[jt]);
    }
}

// C[64 x 64] += A^T B with A, B [16 x 64] row-major in LDS (samples x units):
// C[j][k] = sum_i A[i][j] B[i][k]; acc[rt][ct] holds rows 16 rt.., cols 16 ct..
__device__ inline void wave_gemm_tn(const float *A, const float *B, floatx4 acc[4][4])
{
    const int l = threadIdx.x & 63, i = l & 15, kk = l >> 4;
#pragma unroll
    for (int s = 0; s < ROWS / 4; ++s) {
        float a[4], b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a[t] = A[(4 * s + kk) * H + 16 * t + i];
            b[t] = B[(4 * s + kk) * H + 16 * t + i];
        }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = mfma4(a[rt], b[ct], acc[rt][ct]);
    }
}

// Store a 16 x 64 accumulator (D layout) into LDS row-major, applying f.
template <typename Fn>
__device__ inline void store_acc(float *dstl, const floatx4 acc[4], Fn f)
{
    const int l = threadIdx.x & 63, j = l & 15, i0 = 4 * (l >> 4);
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
        for (int r = 0; r < 4; ++r) dstl[(i0 + r) * H + 16 * jt + j] = f(acc[jt][r], 16 * jt + j, i0 + r);
}

__device__ inline void normalise(const float *x, float z[3])
{
    z[0] = (x[0] - 0.8f) / 0.15f;
    z[1] = (x[1] - 47.5f) / 32.5f;
    z[2] = x[2] - 1.0f;
}

// Forward pass of one wavefront's 16 samples (rows beyond n are zero inputs
// and are masked by the caller).  LDS: h1, h2, h3 [16 x 64] each.  Returns the
// output of sample (l & 15) in every lane of that column group.
__device__ inline void wave_forward(const float *__restrict__ P, const float *__restrict__ X, long row0, long n,
                                    float *h1, float *h2, float *h3, float *yrow)
{
    const int l = threadIdx.x & 63;
    // layer 1 (3 -> 64) on the ALUs: lane l computes units l for all 16 rows
    for (int r = 0; r < ROWS; ++r) {
        const long s = row0 + r;
        float z[3] = {0.f, 0.f, 0.f};
        if (s < n) normalise(X + 3 * s, z);
        const float pre = P[OW1 + 3 * l] * z[0] + P[OW1 + 3 * l + 1] * z[1] + P[OW1 + 3 * l + 2] * z[2] + P[OB1 + l];
        h1[r * H + l] = tanhf(pre);
    }
    __syncthreads();
    floatx4 acc[4];
    for (int jt = 0; jt < 4; ++jt) acc[jt] = floatx4{0.f, 0.f, 0.f, 0.f};
    wave_gemm_16x64(h1, P + OW2, 1, H, acc);  // B(k, j) = W2[j][k]
    store_acc(h2, acc, [&](float v, int j, int) { return tanhf(v + P[OB2 + j]); });
    __syncthreads();
    for (int jt = 0; jt < 4; ++jt) acc[jt] = floatx4{0.f, 0.f, 0.f, 0.f};
    wave_gemm_16x64(h2, P + OW3, 1, H, acc);
    store_acc(h3, acc, [&](float v, int j, int) { return tanhf(v + P[OB3 + j]); });
    __syncthreads();
    // layer 4 (64 -> 1): lane l < 16 sums row l
    if (l < ROWS) {
        float y = P[OB4];
        for (int k = 0; k < H; ++k) y += P[OW4 + k] * h3[l * H + k];
        yrow[l] = y;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(64) k_mlp_forward(const float *__restrict__ P, const float *__restrict__ X,
                                                    float *__restrict__ Y, long n)
{
    __shared__ float h1[ROWS * H], h2[ROWS * H], h3[ROWS * H], yr[ROWS];
    const long row0 = (long)blockIdx.x * ROWS;
    wave_forward(P, X, row0, n, h1, h2, h3, yr);
    const int l = threadIdx.x;
    if (l < ROWS && row0 + l < n) Y[row0 + l] = yr[l];
}

// Forward + backward of the mean squared error for 16 samples; writes this
// wave's partial gradient (NPARAM floats) and partial loss sum.
__global__ void __launch_bounds__(64) k_mlp_grad(const float *__restrict__ P, const float *__restrict__ X,
                                                 const float *__restrict__ Yt, long n, float *__restrict__ G,
                                                 float *__restrict__ Lpart)
{
    __shared__ float h1[ROWS * H], h2[ROWS * H], h3[ROWS * H], dz[ROWS * H], yr[ROWS], dy[ROWS];
    const long row0 = (long)blockIdx.x * ROWS;
    const int l = threadIdx.x;
    wave_forward(P, X, row0, n, h1, h2, h3, yr);
    float *g = G + (long)blockIdx.x * NPARAM;
    if (l < ROWS) {
        const long s = row0 + l;
        const float e = (s < n) ? yr[l] - Yt[s] : 0.f;
        dy[l] = 2.f * e / (float)n;  // d(mean e^2)/dy
        yr[l] = e * e;
    }
    __syncthreads();
    if (l == 0) {
        float sl = 0.f;
        for (int r = 0; r < ROWS; ++r) sl += yr[r];
        Lpart[blockIdx.x] = sl;
    }
    // layer 4: dW4[k] = sum_i dy_i h3[i][k]; db4 = sum_i dy_i; dz3 = dy W4 (1 - h3^2)
    {
        float s = 0.f;
        for (int r = 0; r < ROWS; ++r) s += dy[r] * h3[r * H + l];
        g[OW4 + l] = s;
        if (l == 0) {
            float sb = 0.f;
            for (int r = 0; r < ROWS; ++r) sb += dy[r];
            g[OB4] = sb;
        }
        for (int r = 0; r < ROWS; ++r) {
            const float h = h3[r * H + l];
            dz[r * H + l] = dy[r] * P[OW4 + l] * (1.f - h * h);
        }
    }
    __syncthreads();
    // layers 3 and 2 on the matrix cores
    const float *hin[2] = {h2, h1};
    float *hout[2] = {h3, h2};  // activations whose derivative enters the next dz
    const int ow[2] = {OW3, OW2}, ob[2] = {OB3, OB2};
    for (int layer = 0; layer < 2; ++layer) {
        // dW = dz^T hin, db = sum dz
        floatx4 acc[4][4];
        for (int rt = 0; rt < 4; ++rt)
            for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
        wave_gemm_tn(dz, hin[layer], acc);
        {
            const int j = l & 15, i0 = 4 * (l >> 4);
            for (int rt = 0; rt < 4; ++rt)
                for (int ct = 0; ct < 4; ++ct)
                    for (int r = 0; r < 4; ++r) g[ow[layer] + (16 * rt + i0 + r) * H + 16 * ct + j] = acc[rt][ct][r];
        }
        {
            float sb = 0.f;
            for (int r = 0; r < ROWS; ++r) sb += dz[r * H + l];
            g[ob[layer] + l] = sb;
        }
        // dh_in = dz W (W[j][k]: B(j, k) = W[j * 64 + k]), then dz_in = dh_in (1 - hin^2)
        floatx4 a2[4];
        for (int jt = 0; jt < 4; ++jt) a2[jt] = floatx4{0.f, 0.f, 0.f, 0.f};
        wave_gemm_16x64(dz, P + ow[layer], H, 1, a2);
        __syncthreads();
        const float *hi = hin[layer];
        store_acc(dz, a2, [&](float v, int j, int i) {
            const float h = hi[i * H + j];
            return v * (1.f - h * h);
        });
        __syncthreads();
    }
    (void)hout;
    // layer 1: dW1[k][c] = sum_i dz1[i][k] x_i[c], db1 = sum dz1
    {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, sb = 0.f;
        for (int r = 0; r < ROWS; ++r) {
            const long smp = row0 + r;
            float z[3] = {0.f, 0.f, 0.f};
            if (smp < n) normalise(X + 3 * smp, z);
            const float d = dz[r * H + l];
            s0 += d * z[0];
            s1 += d * z[1];
            s2 += d * z[2];
            sb += d;
        }
        g[OW1 + 3 * l] = s0;
        g[OW1 + 3 * l + 1] = s1;
        g[OW1 + 3 * l + 2] = s2;
        g[OB1 + l] = sb;
    }
}

// Sum the per-wave gradients (fixed order) and apply one Adam step.
__global__ void __launch_bounds__(256) k_mlp_adam(float *__restrict__ P, float *__restrict__ M, float *__restrict__ V,
                                                  const float *__restrict__ G, int nwaves, float *__restrict__ gout,
                                                  int do_update, float lr, float b1, float b2, float eps, float b1t,
                                                  float b2t)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    // fixed summation order; unrolled so that eight partials' loads are in
    // flight at a time instead of one
    float g = 0.f;
#pragma unroll 8
    for (int w = 0; w < nwaves; ++w) g += G[(long)w * NPARAM + p];
    if (gout) gout[p] = g;
    if (!do_update) return;
    const float m = b1 * M[p] + (1.f - b1) * g;
    const float v = b2 * V[p] + (1.f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    const float mh = m / (1.f - b1t), vh = v / (1.f - b2t);
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void __launch_bounds__(64) k_sum_loss(const float *__restrict__ Lpart, int nwaves, long n, float *out)
{
    if (threadIdx.x != 0) return;
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += Lpart[w];
    out[0] = s / (float)n;
}

// Density field of a droplet from the network: rho(x) = rho_c y(T/Tc, R,
// min(|x - c|/R, MLP_RMAX)): beyond r/R = MLP_RMAX, the radial range of the
// training profiles and of the initialiser's probe, the network is not
// evaluated and the far field keeps its value there.
__global__ void __launch_bounds__(64) k_mlp_field(const float *__restrict__ P, int nx, int ny, int nz, double cx,
                                                  double cy, double cz, float R, float Tr, double rho_c,
                                                  double *__restrict__ rho, long n)
{
    __shared__ float h1[ROWS * H], h2[ROWS * H], h3[ROWS * H], yr[ROWS];
    __shared__ float xs[ROWS * 3];
    const long row0 = (long)blockIdx.x * ROWS;
    const int l = threadIdx.x;
    if (l < ROWS) {
        const long c = row0 + l;
        float rr = 0.f;
        if (c < n) {
            const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long)nx * ny));
            const double dx = x - cx, dy = y - cy, dz = nz > 1 ? z - cz : 0.0;
            rr = fminf((float)(sqrt(dx * dx + dy * dy + dz * dz) / R), MLP_RMAX);
        }
        xs[3 * l] = Tr;
        xs[3 * l + 1] = R;
        xs[3 * l + 2] = rr;
    }
    __syncthreads();
    wave_forward(P, xs, 0, ROWS, h1, h2, h3, yr);
    if (l < ROWS && row0 + l < n) rho[row0 + l] = rho_c * (double)yr[l];
}

}  // namespace evlbm

struct evlbm_mlp {
    hipStream_t stream = nullptr;
    float *P = nullptr, *M = nullptr, *V = nullptr;
    float *X = nullptr, *Y = nullptr, *G = nullptr, *L = nullptr, *gsum = nullptr, *loss = nullptr;
    long cap = 0;  // samples the work buffers hold
    long t = 0;    // Adam step count
    // (T/Tc, R) box of the inputs the network was trained on: lo, hi of T/Tc,
    // then of R (empty until trained or set)
    double hull[4] = {HUGE_VAL, -HUGE_VAL, HUGE_VAL, -HUGE_VAL};
};

namespace {

int mlp_reserve(evlbm_mlp *m, long n)
{
    if (n <= m->cap) return EVLBM_OK;
    for (float *p : {m->X, m->Y, m->G, m->L})
        if (p) (void)hipFree(p);
    m->X = m->Y = m->G = m->L = nullptr;
    const long nw = (n + ROWS - 1) / ROWS;
    hipError_t e = hipMalloc(&m->X, sizeof(float) * 3 * n);
    if (e == hipSuccess) e = hipMalloc(&m->Y, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&m->G, sizeof(float) * NPARAM * nw);
    if (e == hipSuccess) e = hipMalloc(&m->L, sizeof(float) * nw);
    if (e != hipSuccess) return fail(EVLBM_ENOMEM, "network work buffers: %s", hipGetErrorString(e));
    m->cap = n;
    return EVLBM_OK;
}

int mlp_upload(evlbm_mlp *m, const float *X, const float *Y, long n)
{
    int rc = mlp_reserve(m, n);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(m->X, X, sizeof(float) * 3 * n, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess && Y) e = hipMemcpyAsync(m->Y, Y, sizeof(float) * n, hipMemcpyHostToDevice, m->stream);
    if (e != hipSuccess) return hip_fail(e, "uploading samples");
    return EVLBM_OK;
}

void launch_grad(evlbm_mlp *m, long n)
{
    const int nw = (int)((n + ROWS - 1) / ROWS);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nw), dim3(64), 0, m->stream, m->P, m->X, m->Y, n, m->G, m->L);
}

}  // namespace

extern "C" {

int evlbm_mlp_create(void *stream, evlbm_mlp_t *out)
{
    if (!out) return fail(EVLBM_EINVAL, "out is NULL");
    evlbm_mlp *m = new evlbm_mlp();
    m->stream = (hipStream_t)stream;
    hipError_t e = hipMalloc(&m->P, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc(&m->M, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc(&m->V, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc(&m->gsum, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMalloc(&m->loss, sizeof(float) * 4);
    if (e == hipSuccess) e = hipMemset(m->P, 0, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMemset(m->M, 0, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMemset(m->V, 0, sizeof(float) * NPARAM);
    if (e != hipSuccess) {
        evlbm_mlp_destroy(m);
        return fail(EVLBM_ENOMEM, "network allocation: %s", hipGetErrorString(e));
    }
    *out = m;
    return EVLBM_OK;
}

int evlbm_mlp_destroy(evlbm_mlp_t m)
{
    if (!m) return EVLBM_OK;
    for (float *p : {m->P, m->M, m->V, m->X, m->Y, m->G, m->L, m->gsum, m->loss})
        if (p) (void)hipFree(p);
    delete m;
    return EVLBM_OK;
}

int evlbm_mlp_num_params(void) { return NPARAM; }

int evlbm_mlp_set_params(evlbm_mlp_t m, const float *params, int n)
{
    if (!m || !params || n != NPARAM) return fail(EVLBM_EINVAL, "need %d parameters", NPARAM);
    hipError_t e = hipMemcpy(m->P, params, sizeof(float) * NPARAM, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->M, 0, sizeof(float) * NPARAM);
    if (e == hipSuccess) e = hipMemset(m->V, 0, sizeof(float) * NPARAM);
    if (e != hipSuccess) return hip_fail(e, "setting parameters");
    m->t = 0;
    return EVLBM_OK;
}

int evlbm_mlp_get_params(evlbm_mlp_t m, float *params, int n)
{
    if (!m || !params || n != NPARAM) return fail(EVLBM_EINVAL, "need %d parameters", NPARAM);
    hipError_t e = hipStreamSynchronize(m->stream);
    if (e == hipSuccess) e = hipMemcpy(params, m->P, sizeof(float) * NPARAM, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading parameters");
    return EVLBM_OK;
}

int evlbm_mlp_forward(evlbm_mlp_t m, const float *X, float *Y, int n)
{
    if (!m || !X || !Y || n <= 0) return fail(EVLBM_EINVAL, "bad arguments");
    int rc = mlp_upload(m, X, nullptr, n);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + ROWS - 1) / ROWS), dim3(64), 0, m->stream, m->P, m->X, m->Y, (long)n);
    hipError_t e = hipMemcpyAsync(Y, m->Y, sizeof(float) * n, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return hip_fail(e, "network forward");
    return EVLBM_OK;
}

int evlbm_mlp_grad(evlbm_mlp_t m, const float *X, const float *Y, int n, float *grad, float *loss)
{
    if (!m || !X || !Y || n <= 0) return fail(EVLBM_EINVAL, "bad arguments");
    int rc = mlp_upload(m, X, Y, n);
    if (rc) return rc;
    launch_grad(m, n);
    const int nw = (n + ROWS - 1) / ROWS;
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->P, m->M, m->V, m->G, nw,
                       m->gsum, 0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f);
    hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, m->stream, m->L, nw, (long)n, m->loss);
    hipError_t e = hipSuccess;
    if (grad) e = hipMemcpyAsync(grad, m->gsum, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return hip_fail(e, "network gradient");
    return EVLBM_OK;
}

int evlbm_mlp_train(evlbm_mlp_t m, const float *X, const float *Y, int n, int iters, float lr, float *loss_hist)
{
    if (!m || !X || !Y || n <= 0 || iters <= 0 || !(lr > 0)) return fail(EVLBM_EINVAL, "bad arguments");
    int rc = mlp_upload(m, X, Y, n);
    if (rc) return rc;
    for (int k = 0; k < n; ++k) {  // the trusted box grows to cover the training inputs
        m->hull[0] = std::fmin(m->hull[0], (double)X[3 * k]);
        m->hull[1] = std::fmax(m->hull[1], (double)X[3 * k]);
        m->hull[2] = std::fmin(m->hull[2], (double)X[3 * k + 1]);
        m->hull[3] = std::fmax(m->hull[3], (double)X[3 * k + 1]);
    }
    const int nw = (n + ROWS - 1) / ROWS;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    std::vector<float> hist(loss_hist ? iters : 0);
    float *dhist = nullptr;
    if (loss_hist) {
        hipError_t e = hipMalloc(&dhist, sizeof(float) * iters);
        if (e != hipSuccess) return fail(EVLBM_ENOMEM, "loss history: %s", hipGetErrorString(e));
    }
    for (int it = 0; it < iters; ++it) {
        launch_grad(m, n);
        if (dhist) hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, m->stream, m->L, nw, (long)n, dhist + it);
        m->t += 1;
        const float b1t = powf(b1, (float)m->t), b2t = powf(b2, (float)m->t);
        hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->P, m->M, m->V, m->G,
                           nw, (float *)nullptr, 1, lr, b1, b2, eps, b1t, b2t);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && dhist)
        e = hipMemcpyAsync(loss_hist, dhist, sizeof(float) * iters, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (dhist) (void)hipFree(dhist);
    if (e != hipSuccess) return hip_fail(e, "network training");
    return EVLBM_OK;
}

int evlbm_mlp_set_hull(evlbm_mlp_t m, double tr_lo, double tr_hi, double r_lo, double r_hi)
{
    if (!m || !(tr_lo <= tr_hi) || !(r_lo <= r_hi)) return fail(EVLBM_EINVAL, "need a network and lo <= hi");
    m->hull[0] = tr_lo;
    m->hull[1] = tr_hi;
    m->hull[2] = r_lo;
    m->hull[3] = r_hi;
    return EVLBM_OK;
}

int evlbm_mlp_get_hull(evlbm_mlp_t m, double out[4])
{
    if (!m || !out) return fail(EVLBM_EINVAL, "null argument");
    for (int k = 0; k < 4; ++k) out[k] = m->hull[k];
    return EVLBM_OK;
}

int evlbm_mlp_density_field(evlbm_mlp_t m, int nx, int ny, int nz, double cx, double cy, double cz, double R,
                            double Tr, double rho_c, double *rho_dev)
{
    if (!m || !rho_dev || nx <= 0 || ny <= 0 || nz <= 0 || !(R > 0)) return fail(EVLBM_EINVAL, "bad arguments");
    const long n = (long)nx * ny * nz;
    hipLaunchKernelGGL(k_mlp_field, dim3((n + ROWS - 1) / ROWS), dim3(64), 0, m->stream, m->P, nx, ny, nz, cx, cy, cz,
                       (float)R, (float)Tr, rho_c, rho_dev, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "network density field");
    return EVLBM_OK;
}

}  // extern "C"

hipStream_t evlbm::mlp_stream(evlbm_mlp_t m) { return m->stream; }
