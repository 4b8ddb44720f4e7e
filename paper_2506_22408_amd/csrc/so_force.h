// so_force.h -- force bias from the mixed Green's function ("Force bias and
// local energy", eq. force_bias with the Cholesky vectors of eq.
// cholesky_vec): xbar_w,gamma = -sqrt(dt) i sum_pq L^gamma_pq G_w,pq.
#pragma once
#include "so_common.h"

// grid (W), 256 threads: G_w (n^2 complex) is staged in LDS, thread t takes
// gamma = t, t + 256, ... and reads L[pq][gamma] (consecutive gamma per warp
// of lanes, coalesced).  n <= SO_NMAX.
__global__ __launch_bounds__(256) void k_force_bias(const double2 *__restrict__ green, int n,
                                                    const double *__restrict__ L, int64_t n_gamma, double sdt,
                                                    double2 *__restrict__ xbar) {
    __shared__ double2 Gs[SO_NMAX * SO_NMAX];
    const int w = blockIdx.x;
    const int nn = n * n;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) Gs[e] = green[(size_t)w * nn + e];
    __syncthreads();
    for (int64_t g = threadIdx.x; g < n_gamma; g += blockDim.x) {
        double ar = 0.0, ai = 0.0;
        for (int e = 0; e < nn; ++e) {
            const double lv = L[(size_t)e * n_gamma + g];
            ar = fma(lv, Gs[e].x, ar);
            ai = fma(lv, Gs[e].y, ai);
        }
        // -sqrt(dt) i (ar + i ai) = sqrt(dt) (ai - i ar)
        xbar[(size_t)w * n_gamma + g] = c_make(sdt * ai, -sdt * ar);
    }
}
