// sampler.hip -- the ensemble sampler step above the likelihood: the
// affine-invariant stretch move of Goodman & Weare (2010) that the paper's
// sampler applies to the walker matrix (Sec. 1 iii; Sec. 3 "Posterior
// sampling"), in its two-half parallel form.  One lane per walker: the
// proposals of a half, then (after the batched likelihood of the proposals)
// their acceptance.  The random numbers are inputs.
#include "internal.hpp"

namespace emri {

// proposals for half h of 2W walkers: partner j = floor(u0 W) of the other
// half, stretch z = ((a - 1) u1 + 1)^2 / a (density ~ 1/sqrt(z) on
// [1/a, a]), Y = X_j + z (X_k - X_j) on the free coordinates; lnz = (D-1) ln z;
// lpr = box log-prior of Y (0 or -inf)
__global__ void __launch_bounds__(256) k_stretch_propose(const double* __restrict__ X, int64_t W,
                                                         int h, PriorBox pr, double a,
                                                         const double* __restrict__ u,
                                                         double* __restrict__ Y,
                                                         double* __restrict__ lnz,
                                                         double* __restrict__ lpr)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= W) return;
    const double* uk = u + 3 * k;
    int64_t j = (int64_t)floor(uk[0] * (double)W);
    j = j < 0 ? 0 : (j > W - 1 ? W - 1 : j);
    const double* xk = X + (h * W + k) * EMRI_NPAR;
    const double* xj = X + ((1 - h) * W + j) * EMRI_NPAR;
    const double s = (a - 1.0) * uk[1] + 1.0;
    const double z = s * s / a;
    double* y = Y + k * EMRI_NPAR;
    for (int i = 0; i < EMRI_NPAR; ++i) y[i] = xk[i];
    bool inside = true;
    for (int d = 0; d < pr.D; ++d) {
        const int i = pr.idx[d];
        y[i] = xj[i] + z * (xk[i] - xj[i]);
        inside = inside && (y[i] >= pr.lo[d] && y[i] <= pr.hi[d]);
    }
    lnz[k] = (double)(pr.D - 1) * log(z);
    lpr[k] = inside ? 0.0 : -INFINITY;
}

// acceptance for half h: lnp(Y) = lpr + lnL; take Y if ln u2 < lnz +
// lnp(Y) - lnp(X_k); a proposal at -inf is rejected, a walker at -inf takes
// any finite proposal
__global__ void __launch_bounds__(256) k_stretch_accept(double* __restrict__ X,
                                                        double* __restrict__ lnp, int64_t W, int h,
                                                        const double* __restrict__ Y,
                                                        const double* __restrict__ lpr,
                                                        const double* __restrict__ lnL,
                                                        const double* __restrict__ lnz,
                                                        const double* __restrict__ u,
                                                        int32_t* __restrict__ acc)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= W) return;
    const int64_t g = h * W + k;
    const double lold = lnp[g], lnew = lpr[k] + lnL[k];
    bool take;
    if (!(lnew > -INFINITY)) take = false;
    else if (!(lold > -INFINITY)) take = true;
    else take = log(u[3 * k + 2]) < lnz[k] + lnew - lold;
    if (take) {
        for (int i = 0; i < EMRI_NPAR; ++i) X[g * EMRI_NPAR + i] = Y[k * EMRI_NPAR + i];
        lnp[g] = lnew;
    }
    if (acc) acc[g] = take ? 1 : 0;
}

// lnp[k] += box log-prior of X_k
__global__ void __launch_bounds__(256) k_add_box_prior(const double* __restrict__ X, int64_t n,
                                                       PriorBox pr, double* __restrict__ lnp)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double* x = X + k * EMRI_NPAR;
    bool inside = true;
    for (int d = 0; d < pr.D; ++d) {
        const double v = x[pr.idx[d]];
        inside = inside && (v >= pr.lo[d] && v <= pr.hi[d]);
    }
    if (!inside) lnp[k] = -INFINITY;
}

hipError_t launch_stretch_propose(const double* X, int64_t W, int h, const PriorBox& pr, double a,
                                  const double* u, double* Y, double* lnz, double* lpr,
                                  hipStream_t s)
{
    trace_mark(ST_SAMPLER, s, true);
    hipLaunchKernelGGL(k_stretch_propose, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, s, X,
                       W, h, pr, a, u, Y, lnz, lpr);
    trace_mark(ST_SAMPLER, s, false);
    return hipGetLastError();
}

hipError_t launch_stretch_accept(double* X, double* lnp, int64_t W, int h, const double* Y,
                                 const double* lpr, const double* lnL, const double* lnz,
                                 const double* u, int32_t* acc, hipStream_t s)
{
    trace_mark(ST_SAMPLER, s, true);
    hipLaunchKernelGGL(k_stretch_accept, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, s, X,
                       lnp, W, h, Y, lpr, lnL, lnz, u, acc);
    trace_mark(ST_SAMPLER, s, false);
    return hipGetLastError();
}

hipError_t launch_add_box_prior(const double* X, int64_t n, const PriorBox& pr, double* lnp,
                                hipStream_t s)
{
    trace_mark(ST_SAMPLER, s, true);
    hipLaunchKernelGGL(k_add_box_prior, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, n,
                       pr, lnp);
    trace_mark(ST_SAMPLER, s, false);
    return hipGetLastError();
}

}  // namespace emri
