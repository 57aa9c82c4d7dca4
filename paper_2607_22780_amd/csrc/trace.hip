// trace.hip -- Trace(r_o, r_d) forward and its backward by re-traversal.
//
// Forward (Sec. 3.2, Eq. trace): the hits of a ray arrive from the ordered
// traversal in ascending (tau, id); each one composites
//   C += T alpha c,  T <- T (1 - alpha),  alpha = o exp(-rho^2 / 2)
// until T < t_cut (that hit included).  Returns c_rt = C and T = 1 - o_rt.
//
// Backward: with the forward's C and T_fin known, the same traversal
// replays the hits in the same order and, per hit k,
//   dL/dc_k     = T_k alpha_k g_C
//   dL/dalpha_k = T_k (g_C . c_k) - [g_C . (C - P_k) + g_T T_fin] / (1 - alpha_k)
// (P_k = colour composited through hit k), then chains alpha -> (o, u, v)
// -> (s_u, s_v, mu, t_u, t_v, n) -> q, and adds the 13 parameter gradients of
// the surfel with device atomics.
#include "grt_internal.h"
#include "grt_kernels.h"

namespace grt {

template <int K>
__global__ void __launch_bounds__(256) k_trace(TraceArgs a)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    const float3 o = make_float3(a.o[3 * r], a.o[3 * r + 1], a.o[3 * r + 2]);
    const float3 d = make_float3(a.d[3 * r], a.d[3 * r + 1], a.d[3 * r + 2]);
    const float tmin = a.tmin_a ? a.tmin_a[r] : a.tmin;
    const float tmax = a.tmax_a ? a.tmax_a[r] : a.tmax;
    CompositeVisit v(a.S, o, d, a.tcut);
    if (a.dump_id) { v.did = a.dump_id + r * a.cap; v.dtau = a.dump_tau + r * a.cap; v.cap = a.cap; }
    traverse<K>(a.S, o, d, tmin, tmax, v);
    a.out_rgb[3 * r] = v.C.x; a.out_rgb[3 * r + 1] = v.C.y; a.out_rgb[3 * r + 2] = v.C.z;
    a.out_T[r] = v.T;
    if (a.out_L) {
        a.out_L[3 * r] = v.C.x + v.T * a.sky[0];
        a.out_L[3 * r + 1] = v.C.y + v.T * a.sky[1];
        a.out_L[3 * r + 2] = v.C.z + v.T * a.sky[2];
    }
    if (a.out_nhit) a.out_nhit[r] = v.cnt;
    if (a.dump_id) {
        for (int i = v.cnt; i < a.cap; ++i) { v.did[i] = -1; v.dtau[i] = 0.0f; }
    }
}

template <int K>
__global__ void __launch_bounds__(256) k_trace_bwd(TraceBwdArgs a)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.f.n) return;
    const float3 o = make_float3(a.f.o[3 * r], a.f.o[3 * r + 1], a.f.o[3 * r + 2]);
    const float3 d = make_float3(a.f.d[3 * r], a.f.d[3 * r + 1], a.f.d[3 * r + 2]);
    const float tmin = a.f.tmin_a ? a.f.tmin_a[r] : a.f.tmin;
    const float tmax = a.f.tmax_a ? a.f.tmax_a[r] : a.f.tmax;
    const float3 gC = make_float3(a.grad_rgb[3 * r], a.grad_rgb[3 * r + 1], a.grad_rgb[3 * r + 2]);
    const float gT = a.grad_T ? a.grad_T[r] : 0.0f;
    if (gC.x == 0.0f && gC.y == 0.0f && gC.z == 0.0f && gT == 0.0f) return;
    const float3 C = make_float3(a.fwd_rgb[3 * r], a.fwd_rgb[3 * r + 1], a.fwd_rgb[3 * r + 2]);
    GradVisit v(a.f.S, a.f.tcut, a.g, o, d, gC, gT, C, a.fwd_T[r]);
    traverse<K>(a.f.S, o, d, tmin, tmax, v);
}

hipError_t launch_trace(const TraceArgs &a, int k, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    switch (k) {
    case 1: hipLaunchKernelGGL(k_trace<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_trace<2>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_trace<4>, grid, block, 0, st, a); break;
    case 8: hipLaunchKernelGGL(k_trace<8>, grid, block, 0, st, a); break;
    case 16: hipLaunchKernelGGL(k_trace<16>, grid, block, 0, st, a); break;
    case 32: hipLaunchKernelGGL(k_trace<32>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_trace_backward(const TraceBwdArgs &a, int k, hipStream_t st)
{
    if (a.f.n <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.f.n + 255) / 256)), block(256);
    switch (k) {
    case 1: hipLaunchKernelGGL(k_trace_bwd<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_trace_bwd<2>, grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_trace_bwd<4>, grid, block, 0, st, a); break;
    case 8: hipLaunchKernelGGL(k_trace_bwd<8>, grid, block, 0, st, a); break;
    case 16: hipLaunchKernelGGL(k_trace_bwd<16>, grid, block, 0, st, a); break;
    case 32: hipLaunchKernelGGL(k_trace_bwd<32>, grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace grt
