// Library-internal state shared by the lattice, batch and network sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "evlbm.h"

struct evlbm_lattice {
    int D = 2, Q = 9, nx = 0, ny = 0, nz = 0, storage = EVLBM_F32;
    long N = 0;
    long ds = 0;                        // direction stride of the population buffers (elements)
    int device = 0;
    hipStream_t stream = nullptr;
    void *buf[2] = {nullptr, nullptr};  // population buffers, f then g: 2Q arrays of N cells, ds apart
    bool own_buf = true;                // false once the caller attached its own population buffers
    int cur = 0;                        // buffer holding the current state
    void *m = nullptr;                  // pulled moments rho, j (D), e: [(D+2)][N] of the current state
    void *m_alt = nullptr;              // D3Q27 one-pass step: the next state's moments (swapped with m)
    void *shell = nullptr;              // D3Q27 one-pass step: partial moment sums around each tile chunk
    void *lap = nullptr;                // readout scratch: lap rho [N]
    float4 *refst = nullptr;            // 16-bit deviation storage: reference state per cell [N]
    void *scratch = nullptr;            // I/O and reduction scratch
    size_t scratch_bytes = 0;
    // model
    double R = 1.0, a = 0.0, b = 0.0, kappa = 0.0, tau = 1.0, lambda = 1.0, sphi = -1.0;
    int eos = EVLBM_EOS_VDW;
    double prandtl = 1.0;               // Pr = tau/tau_g of the energy populations
    // diffuse walls normal to x (evlbm_set_walls): temperature, speed of the
    // wall at x = nx - 1/2, work buffers of the wall step (streamed
    // populations [2Q][N], fields [3D + 2][N], arithmetic precision)
    bool walls = false;
    double Tw = 0.0, Uw = 0.0;
    void *wall_fh = nullptr, *wall_fld = nullptr;
    int64_t check_every = 0;
    int64_t reref_every = 100;           // 16-bit storage: re-reference period (0 = never)
    bool use_graph = true;
    bool push = true;                    // D3Q27: moments pushed by the collision (one-pass step)
    // state
    int64_t step = 0;
    bool initialized = false;
    bool m_valid = false;
    hipGraphExec_t graph_exec_par[2] = {nullptr, nullptr};  // captured step chunks, per buffer parity
};

namespace evlbm {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int ensure_scratch(evlbm_lattice *h, size_t bytes);
void refresh_moments(evlbm_lattice *h);
void launch_step(evlbm_lattice *h, hipEvent_t between = nullptr);
int run_steps(evlbm_lattice *h, int64_t n);
int scan_nonfinite(evlbm_lattice *h);
int rereference(evlbm_lattice *h);
size_t store_bytes(int storage);
hipStream_t mlp_stream(evlbm_mlp_t m);  // the stream a network's kernels run on
// largest r/R the network's density field evaluates it at (the radial range
// of its training profiles and of the droplet initialiser's probe)
constexpr float MLP_RMAX = 3.0f;
// the wall step and its readouts (evlbm_walls.hip)
void wall_step(evlbm_lattice *h);
void wall_analyse(evlbm_lattice *h);
int wall_read_moments(evlbm_lattice *h, void *rho, void *u, void *T, int where, double *host_scratch);
void wall_sums(evlbm_lattice *h, double *partial);
size_t real_bytes(int storage);

}  // namespace evlbm
