// tempering.hip -- one parallel-tempering pass per (sample, replica).
//
// Appendix A.1: a swap of the configurations at neighbouring temperatures is
// proposed for each pair of slots and accepted with the Metropolis
// probability; exchanging configurations is the same as exchanging their
// temperatures, so only the slot labels (perm, slot_of, beta_of) change and
// no spin moves.  The pairs are visited in ascending order within a pass,
// which makes the pass sequential per (sample, replica): one lane each.
#include <algorithm>

#include "kernels.hpp"
#include "philox.hpp"

namespace ptsg {

namespace {

// The pass of ladder t = (sample, replica).
__device__ void swap_ladder(const SwapParams &P, int t, uint32_t pass)
{
    const int s = t / P.R;
    const int r = t - s * P.R;
    const int T = P.n_temps[s];
    int *perm = P.perm + P.perm_base[s] + r * T;
    const double *beta = P.betas + P.beta_base[s];
    const int cb = P.chain_base[s] + r * T;
    const double *E = P.E + cb;
    // The configuration that moves up the ladder is carried in registers
    // (its chain a and energy ea): slot k + 1 still holds its value from
    // before the pass when pair (k, k+1) is decided, and slot k is final
    // once it is, so every load is independent of the decisions and each
    // slot is written once.
    int a = perm[0];
    double ea = E[a];
    for (int k = 0; k + 1 < T; ++k) {
        const int b = perm[k + 1];
        const double eb = E[b];
        const double delta = (beta[k] - beta[k + 1]) * (ea - eb);
        const uint4 w = philox10(make_uint4(static_cast<uint32_t>(k), pass,
                                            static_cast<uint32_t>(s),
                                            ctr_word3(1u, 0u, static_cast<uint32_t>(r))),
                                 P.key0, P.key1);
        const bool swap = delta >= 0.0 || unit52(w.x, w.y) < exp(delta);
        const int stay = swap ? b : a;   // the configuration left at slot k
        perm[k] = stay;
        P.slot_of[cb + stay] = k;
        P.beta_of[cb + stay] = static_cast<float>(beta[k]);
        if (!swap) {
            a = b;
            ea = eb;
        }
    }
    perm[T - 1] = a;
    P.slot_of[cb + a] = T - 1;
    P.beta_of[cb + a] = static_cast<float>(beta[T - 1]);
}

// One workgroup: thread t takes ladders t, t + blockDim.x, ...; after the
// barrier, when every thread has read the pass counter, thread 0 advances
// it (no separate launch for the counter).
__global__ __launch_bounds__(1024) void swap_kernel(SwapParams P)
{
    const uint32_t pass = P.counters[1];
    const int n = P.n_samples * P.R;
    for (int t = static_cast<int>(threadIdx.x); t < n; t += static_cast<int>(blockDim.x))
        swap_ladder(P, t, pass);
    __syncthreads();
    if (threadIdx.x == 0) P.counters[1] = pass + 1u;
}

}  // namespace

hipError_t launch_swap(const SwapParams &p, hipStream_t st)
{
    const int n = p.n_samples * p.R;
    const int block = std::min(1024, std::max(64, (n + 63) / 64 * 64));
    hipLaunchKernelGGL(swap_kernel, dim3(1), dim3(block), 0, st, p);
    return hipGetLastError();
}

}  // namespace ptsg
