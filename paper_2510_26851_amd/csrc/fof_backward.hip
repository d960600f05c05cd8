// Frozen-assignment backward (paper Sec. 3.1 and its differentiation-modes table):
// memberships stay as the forward found them; the group position is the mean member
// position, so d com_g / d x_i = 1/n_g for members; the member count (mass) has zero
// gradient; the velocity dispersion sigma = sqrt(sum (v - vbar)^2 / (3 n)) gives
// d sigma / d v_ic = (v_ic - vbar_c) / (3 n sigma).  One thread per particle, a gather of
// its group's upstream gradients; FP64 arithmetic, FP32 outputs.
#include "fof_internal.h"

namespace fof {

namespace {

__global__ void k_frozen_bwd(int64_t n, const int32_t *__restrict__ group_id, int32_t G,
                             const int32_t *__restrict__ sizes, const double *__restrict__ vmean,
                             const double *__restrict__ sigv, const float *__restrict__ vel,
                             const double *__restrict__ g_com, const double *__restrict__ g_sigv,
                             float *__restrict__ grad_pos, float *__restrict__ grad_vel)
{
    const int64_t i = gtid();
    if (i >= n)
        return;
    const int32_t g = group_id[i];
    const bool in = g >= 0 && g < G;
    double gp[3] = {0.0, 0.0, 0.0}, gv[3] = {0.0, 0.0, 0.0};
    if (in) {
        const double dn = (double)sizes[g];
        if (g_com)
            for (int a = 0; a < 3; ++a)
                gp[a] = g_com[3 * g + a] / dn;
        if (grad_vel && g_sigv && sigv[g] > 0.0) {
            const double f = g_sigv[g] / (3.0 * dn * sigv[g]);
            for (int a = 0; a < 3; ++a)
                gv[a] = f * ((double)vel[3 * i + a] - vmean[3 * g + a]);
        }
    }
    if (grad_pos)
        for (int a = 0; a < 3; ++a)
            grad_pos[3 * i + a] = (float)gp[a];
    if (grad_vel)
        for (int a = 0; a < 3; ++a)
            grad_vel[3 * i + a] = (float)gv[a];
}

}  // namespace

hipError_t launch_backward(int64_t n, int32_t block, const int32_t *group_id, int32_t G,
                           const int32_t *sizes, const double *vmean, const double *sigv,
                           const float *vel, const double *g_com, const double *g_sigv,
                           float *grad_pos, float *grad_vel, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const unsigned nb = (unsigned)((n + block - 1) / block);
    hipLaunchKernelGGL(k_frozen_bwd, dim3(nb), dim3(block), 0, s, n, group_id, G, sizes, vmean,
                       sigv, vel, g_com, g_sigv, grad_pos, grad_vel);
    return hipGetLastError();
}

}  // namespace fof
