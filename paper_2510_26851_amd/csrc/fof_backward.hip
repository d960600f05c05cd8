// Frozen-assignment backward (paper Sec. 3.1 and its differentiation-modes table), and the
// gradient of the position-dispersion decoration (decorated frozen assignment):
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

// Decorated frozen assignment (Sec. 3.1): the position dispersion
// sigx = sqrt(sum_i |mi(x_i - com)|^2 / (3 n)), mi the per-axis minimum image, has
// d sigx / d x_ic = mi(x_ic - com_c) / (3 n sigx) (the com terms cancel: the deviations
// sum to zero).  Adds g_sigx[g] times that to grad_pos.
__global__ void k_sigx_bwd(int64_t n, const BoxDesc *__restrict__ desc, int nbox,
                           const float *__restrict__ pos, const int32_t *__restrict__ group_id,
                           int32_t G, const int32_t *__restrict__ sizes,
                           const double *__restrict__ com, const double *__restrict__ sigx,
                           const double *__restrict__ g_sigx, float *__restrict__ grad_pos)
{
    const int64_t i = gtid();
    if (i >= n)
        return;
    const int32_t g = group_id[i];
    if (g < 0 || g >= G || !(sigx[g] > 0.0))
        return;
    const BoxDesc &B = desc[find_box(desc, nbox, i)];
    const double f = g_sigx[g] / (3.0 * (double)sizes[g] * sigx[g]);
    for (int a = 0; a < 3; ++a) {
        const double x = (double)pos[3 * i + a];
        const double d = min_image(x - com[3 * g + a], B.L[a], B.halfL[a]);
        grad_pos[3 * i + a] += (float)(f * d);
    }
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

hipError_t launch_backward_dispersion(const Work &w, const float *pos, const int32_t *group_id,
                                      int32_t G, const int32_t *sizes, const double *com,
                                      const double *sigx, const double *g_sigx, float *grad_pos,
                                      hipStream_t s)
{
    if (w.n <= 0 || G <= 0)
        return hipSuccess;
    const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
    hipLaunchKernelGGL(k_sigx_bwd, dim3(nb), dim3(w.block), 0, s, w.n, w.desc, w.nbox, pos,
                       group_id, G, sizes, com, sigx, g_sigx, grad_pos);
    return hipGetLastError();
}

}  // namespace fof
