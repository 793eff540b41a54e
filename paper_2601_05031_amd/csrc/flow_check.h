// Convergence check of the two flow solves of a step, each of a single cycle (main text
// eq. (5b), (5c); the solves are verified against a relative-residual tolerance). Partial
// slots 0-5 hold the vorticity residual sums, 6-11 the stream-vector ones (per component,
// value-major: r^2 in slots 0-2, b~^2 in 3-5); the two checks run in a row (vorticity, then
// stream vector) as two last-cycle checks would. Shared by the standalone check kernel and by
// the first block of the next step's advance, which takes the check of the previous step.
#pragma once
#include "vs_internal.h"

namespace vs {

__device__ __forceinline__ double fc_wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Call from every thread of one block (a multiple of 64 threads, at most 1024); sh holds
// 4 * 16 doubles. last_cycle = 0 (a defect-correction cycle that may be followed by another):
// the convergence flag gates the next cycle and the miss is not yet an error. log (or null):
// the step's final check (converged, or the last cycle) appends a record to the per-step log.
__device__ inline void flow_check_block(const double* __restrict__ partials, int nblocks,
                                        double rtol, double* scal, int* istat, double* sh,
                                        int last_cycle = 1, double* log = nullptr) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const double* pb = partials + (size_t)(3 * g) * kMaxPartialBlocks + b;
            a[g] += pb[0] + pb[kMaxPartialBlocks] + pb[2 * kMaxPartialBlocks];
        }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) a[g] = fc_wave_sum(a[g]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int g = 0; g < 4; ++g) sh[g * 16 + wv] = a[g];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int g = 0; g < 4; ++g) {
            a[g] = 0.0;
            for (int q = 0; q < nw; ++q) a[g] += sh[g * 16 + q];
        }
        double rel[2];
        int conv = 1;
        for (int sidx = 0; sidx < 2; ++sidx) {
            const double rr = a[2 * sidx], bb = a[2 * sidx + 1];
            double r;
            if (bb > 0.0)
                r = sqrt(rr / bb);
            else
                r = (rr > 0.0) ? INFINITY : 0.0;
            if (rr != rr || bb != bb) r = NAN;
            rel[sidx] = r;
            conv &= (r <= rtol) ? 1 : 0;
            istat[IS_CYCLES] += 1;
            scal[SC_RELRES_LAST] = r;
            if (!isfinite(rr) || !isfinite(bb)) istat[IS_FLAGS] |= ST_NONFINITE;
        }
        istat[IS_CONV] = conv;
        if (conv || last_cycle) {
            for (int sidx = 0; sidx < 2; ++sidx) {
                const double prev = scal[SC_RELRES_MAX];
                scal[SC_RELRES_MAX] = (rel[sidx] != rel[sidx] || rel[sidx] > prev) ? rel[sidx] : prev;
            }
            if (log) {
                const int n = istat[IS_LOGN];
                double* r = log + (size_t)(n % kLogCap) * kLogFields;
                r[0] = (double)n;
                r[1] = (double)istat[IS_CYCLES];
                r[2] = (rel[0] != rel[0] || rel[0] > rel[1]) ? rel[0] : rel[1];
                r[3] = scal[SC_V];
                r[4] = scal[SC_A];
                r[5] = scal[SC_LAMV];
                r[6] = scal[SC_GAMMA];
                r[7] = (double)(conv ? 1 : 0);
                istat[IS_LOGN] = n + 1;
            }
        }
        if (!conv && last_cycle) istat[IS_FLAGS] |= ST_NOCONV;
    }
    __syncthreads();
}

}  // namespace vs
