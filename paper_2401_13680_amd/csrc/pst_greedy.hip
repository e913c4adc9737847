// Snippet selection on the profile set D, entirely on device.
//
//   - greedy minimum-area search (section 4.1, eqs. 16-17): K rounds; in each,
//     every unchosen segment's area sum_j min(M_j, D_s(j)) is summed in FP64 in
//     a fixed order (per-block tree sums, then blocks in order), the smallest
//     area wins with ties to the lowest segment index, and M <- min(M, D_pick);
//   - neighbours and frac (eqs. 6-7): each window is owned by the chosen
//     snippet with the smallest profile value there, ties to the earlier pick;
//   - the snippet-length criterion numerator (eq. 18): sum over ordered pairs
//     of picked profiles of sum_j |D_p(j) - D_q(j)|.
#include "pst_internal.h"

#include <math.h>

namespace pst {
namespace {

constexpr int GT = 256;

__global__ void k_fill(float *__restrict__ p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < n; i += (int64_t)gridDim.x * GT)
        p[i] = v;
}

__global__ void k_zero_u8(uint8_t *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < n; i += (int64_t)gridDim.x * GT)
        p[i] = 0;
}

__global__ void k_set_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < n; i += (int64_t)gridDim.x * GT)
        p[i] = v;
}

__global__ void k_zero_i32(int32_t *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < n; i += (int64_t)gridDim.x * GT)
        p[i] = 0;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int o = GT / 2; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// part[s * nblk + b] = sum over block b's windows of min(M_j, D_s(j)).
__global__ void __launch_bounds__(GT) k_area_part(GreedyJob g) {
    __shared__ double red[GT];
    const int s = blockIdx.y, b = blockIdx.x;
    if (g.chosen[s]) return;
    const int64_t j0 = (int64_t)b * kSumBlock;
    const int64_t j1 = j0 + kSumBlock < g.Nm ? j0 + kSumBlock : g.Nm;
    const float *Ds = g.D + (int64_t)s * g.ld;
    double acc = 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += GT) acc += (double)fminf(g.M[j], Ds[j]);
    double tot = block_sum(acc, red);
    if (threadIdx.x == 0) g.part[(int64_t)s * g.nblk + b] = tot;
}

// One block: smallest area among unchosen segments, ties to the lowest index.
__global__ void __launch_bounds__(1024) k_pick(GreedyJob g, int iter) {
    __shared__ double ra[1024];
    __shared__ int rs[1024];
    const int t = threadIdx.x;
    double best = INFINITY;
    int bs = 0x7fffffff;
    for (int s = t; s < g.nseg; s += 1024) {
        if (g.chosen[s]) continue;
        double a = 0.0;
        const double *p = g.part + (int64_t)s * g.nblk;
        for (int b = 0; b < g.nblk; ++b) a += p[b];
        if (a < best || (a == best && s < bs)) {
            best = a;
            bs = s;
        }
    }
    ra[t] = best;
    rs[t] = bs;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) {
            const double a2 = ra[t + o];
            const int s2 = rs[t + o];
            if (a2 < ra[t] || (a2 == ra[t] && s2 < rs[t])) {
                ra[t] = a2;
                rs[t] = s2;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        g.pick[iter] = rs[0];
        g.area[iter] = ra[0];
        g.chosen[rs[0]] = 1;
    }
}

__global__ void k_update_M(GreedyJob g, int iter) {
    const float *Dp = g.D + (int64_t)g.pick[iter] * g.ld;
    for (int64_t j = (int64_t)blockIdx.x * GT + threadIdx.x; j < g.Nm; j += (int64_t)gridDim.x * GT)
        g.M[j] = fminf(g.M[j], Dp[j]);
}

__global__ void __launch_bounds__(GT) k_owner(GreedyJob g) {
    extern __shared__ int cnt_lds[];
    const bool use_lds = g.K <= 1024;
    if (use_lds) {
        for (int p = threadIdx.x; p < g.K; p += GT) cnt_lds[p] = 0;
        __syncthreads();
    }
    for (int64_t j = (int64_t)blockIdx.x * GT + threadIdx.x; j < g.Nm; j += (int64_t)gridDim.x * GT) {
        float best = g.D[(int64_t)g.pick[0] * g.ld + j];
        int bp = 0;
        for (int p = 1; p < g.K; ++p) {
            const float v = g.D[(int64_t)g.pick[p] * g.ld + j];
            if (v < best) {
                best = v;
                bp = p;
            }
        }
        if (g.owner) g.owner[j] = bp;
        if (use_lds) atomicAdd(&cnt_lds[bp], 1);
        else atomicAdd(&g.count[bp], 1);
        if (g.profiles)
            for (int p = 0; p < g.K; ++p)
                g.profiles[(int64_t)p * g.Nm + j] = g.D[(int64_t)g.pick[p] * g.ld + j];
    }
    if (use_lds) {
        __syncthreads();
        for (int p = threadIdx.x; p < g.K; p += GT)
            if (cnt_lds[p]) atomicAdd(&g.count[p], cnt_lds[p]);
    }
}

__global__ void __launch_bounds__(GT) k_crit_part(GreedyJob g) {
    __shared__ double red[GT];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * GT + threadIdx.x; j < g.Nm; j += (int64_t)gridDim.x * GT) {
        for (int p = 0; p < g.K; ++p) {
            const float a = g.D[(int64_t)g.pick[p] * g.ld + j];
            for (int q = p + 1; q < g.K; ++q)
                acc += fabs((double)a - (double)g.D[(int64_t)g.pick[q] * g.ld + j]);
        }
    }
    double tot = block_sum(acc, red);
    if (threadIdx.x == 0) g.crit[blockIdx.x] = tot;
}

__global__ void k_crit_final(GreedyJob g) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < g.nblk2; ++b) s += g.crit[b];
    g.crit[g.nblk2] = 2.0 * s;  // ordered pairs p != q
}

__global__ void k_gather(SweepGather G) {
    const int stride = 3 + 3 * G.K;
    for (int i = threadIdx.x; i < G.nm * stride; i += blockDim.x) {
        const int c = i / stride, e = i - c * stride;
        double v;
        if (e == 0) v = *G.crit[c];
        else if (e == 1) v = (double)*G.dmax[c];
        else if (e == 2) v = *G.bad[c];
        else if (e < 3 + G.K) v = G.area[c][e - 3];
        else if (e < 3 + 2 * G.K) v = (double)G.pick[c][e - 3 - G.K];
        else v = (double)G.count[c][e - 3 - 2 * G.K];
        G.out[i] = v;
    }
}

inline int grid_for(int64_t n) {
    int64_t b = (n + GT - 1) / GT;
    return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_u32, dim3(grid_for(n)), dim3(GT), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_greedy(const GreedyJob &g, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(g.Nm)), dim3(GT), 0, st, g.M, g.Nm, INFINITY);
    hipLaunchKernelGGL(k_zero_u8, dim3(grid_for(g.nseg)), dim3(GT), 0, st, g.chosen, (int64_t)g.nseg);
    for (int it = 0; it < g.K; ++it) {
        hipLaunchKernelGGL(k_area_part, dim3(g.nblk, g.nseg), dim3(GT), 0, st, g);
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(1024), 0, st, g, it);
        hipLaunchKernelGGL(k_update_M, dim3(grid_for(g.Nm)), dim3(GT), 0, st, g, it);
    }
    return hipGetLastError();
}

hipError_t launch_greedy_init(const GreedyJob &g, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(g.Nm)), dim3(GT), 0, st, g.M, g.Nm, INFINITY);
    hipLaunchKernelGGL(k_zero_u8, dim3(grid_for(g.nseg)), dim3(GT), 0, st, g.chosen, (int64_t)g.nseg);
    return hipGetLastError();
}

hipError_t launch_area_parts(const GreedyJob &g, hipStream_t st) {
    hipLaunchKernelGGL(k_area_part, dim3(g.nblk, g.nseg), dim3(GT), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_pick(const GreedyJob &g, int iter, hipStream_t st) {
    hipLaunchKernelGGL(k_pick, dim3(1), dim3(1024), 0, st, g, iter);
    return hipGetLastError();
}

hipError_t launch_update_M(const GreedyJob &g, int iter, hipStream_t st) {
    hipLaunchKernelGGL(k_update_M, dim3(grid_for(g.Nm)), dim3(GT), 0, st, g, iter);
    return hipGetLastError();
}

hipError_t launch_owner(const GreedyJob &g, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(g.K)), dim3(GT), 0, st, g.count, (int64_t)g.K);
    const size_t lds = g.K <= 1024 ? sizeof(int) * g.K : 0;
    hipLaunchKernelGGL(k_owner, dim3(grid_for(g.Nm)), dim3(GT), lds, st, g);
    return hipGetLastError();
}

hipError_t launch_gather(const SweepGather &g, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(1), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_criterion(const GreedyJob &g, hipStream_t st) {
    hipLaunchKernelGGL(k_crit_part, dim3(g.nblk2), dim3(GT), 0, st, g);
    hipLaunchKernelGGL(k_crit_final, dim3(1), dim3(64), 0, st, g);
    return hipGetLastError();
}

}  // namespace pst
