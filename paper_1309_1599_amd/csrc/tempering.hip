// tempering.hip -- one parallel-tempering pass per (sample, replica).
//
// Appendix A.1: a swap of the configurations at neighbouring temperatures is
// proposed for each pair of slots and accepted with the Metropolis
// probability; exchanging configurations is the same as exchanging their
// temperatures, so only the slot labels (perm, slot_of, beta_of) change and
// no spin moves.  The pairs are visited in ascending order within a pass,
// which makes the pass sequential per (sample, replica): one lane each.
#include "kernels.hpp"
#include "philox.hpp"

namespace ptsg {

namespace {

__global__ void swap_kernel(SwapParams P)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.n_samples * P.R) return;
    const int s = t / P.R;
    const int r = t - s * P.R;
    const int T = P.n_temps[s];
    int *perm = P.perm + P.perm_base[s] + r * T;
    const double *beta = P.betas + P.beta_base[s];
    const int cb = P.chain_base[s] + r * T;
    const double *E = P.E + cb;
    const uint32_t pass = P.counters[1];
    for (int k = 0; k + 1 < T; ++k) {
        const int a = perm[k], b = perm[k + 1];
        const double delta = (beta[k] - beta[k + 1]) * (E[a] - E[b]);
        const uint4 w = philox10(make_uint4(static_cast<uint32_t>(k), pass,
                                            static_cast<uint32_t>(s),
                                            ctr_word3(1u, 0u, static_cast<uint32_t>(r))),
                                 P.key0, P.key1);
        if (delta >= 0.0 || unit52(w.x, w.y) < exp(delta)) {
            perm[k] = b;
            perm[k + 1] = a;
        }
    }
    for (int k = 0; k < T; ++k) {
        const int chain = cb + perm[k];
        P.slot_of[chain] = k;
        P.beta_of[chain] = static_cast<float>(beta[k]);
    }
}

}  // namespace

hipError_t launch_swap(const SwapParams &p, hipStream_t st)
{
    const int n = p.n_samples * p.R;
    hipLaunchKernelGGL(swap_kernel, dim3((n + 63) / 64), dim3(64), 0, st, p);
    return hipGetLastError();
}

}  // namespace ptsg
