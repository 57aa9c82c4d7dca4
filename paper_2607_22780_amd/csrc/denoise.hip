// denoise.hip -- cross-bilateral denoiser for low-sample renders (Sec. 3.4.2,
// "Denoising"; SVGF-style spatial filtering guided by depth and normal).
//
// For each valid pixel p, over the valid pixels p' of the (2R+1)^2 window:
//   B(p,p') = exp(-|p-p'|^2 / (2 sigma_s^2))
//           * exp(-|D(p)-D(p')| / (sigma_d |grad D(p) . (p-p')| + eps_d))
//           * max(0, N(p).N(p'))^sigma_n
//   out(p)  = sum B c(p') / sum B
// N is normalized per pixel; grad D is the screen-space depth gradient by
// central differences (one-sided where a neighbour is outside the image or
// invalid, 0 where both are).  Invalid pixels pass through unchanged.
//
// Image-space stencil: a workgroup stages its 16x16 pixels and an R-pixel
// halo (colour, depth, unit normal, validity) in LDS once, so each input is
// read from HBM about (16+2R)^2/256 times instead of (2R+1)^2 times.
#include "grt_internal.h"

namespace grt {

constexpr int kDnTile = 16;
constexpr int kDnSpan = kDnTile + 2 * kDenoiseMaxRadius;

__global__ void __launch_bounds__(256) k_denoise(DenoiseArgs a)
{
    __shared__ float4 lc[kDnSpan * kDnSpan];  // rgb, depth
    __shared__ float4 ln[kDnSpan * kDnSpan];  // unit normal, valid (1/0)
    const int R = a.radius, span = kDnTile + 2 * R;
    const int x0 = blockIdx.x * kDnTile - R, y0 = blockIdx.y * kDnTile - R;
    for (int i = threadIdx.x; i < span * span; i += blockDim.x) {
        const int ty = i / span, tx = i - ty * span;
        const int gx = x0 + tx, gy = y0 + ty;
        float4 c = make_float4(0.f, 0.f, 0.f, 0.f), n = c;
        if (gx >= 0 && gx < a.W && gy >= 0 && gy < a.H) {
            const int64_t p = (int64_t)gy * a.W + gx;
            if (a.valid[p]) {
                const float nx = a.normal[3 * p], ny = a.normal[3 * p + 1], nz = a.normal[3 * p + 2];
                const float l = sqrtf(nx * nx + ny * ny + nz * nz);
                const float il = l > 0.0f ? 1.0f / l : 0.0f;
                c = make_float4(a.rgb[3 * p], a.rgb[3 * p + 1], a.rgb[3 * p + 2], a.depth[p]);
                n = make_float4(nx * il, ny * il, nz * il, 1.0f);
            }
        }
        lc[ty * span + tx] = c;
        ln[ty * span + tx] = n;
    }
    __syncthreads();
    const int tx = threadIdx.x % kDnTile, ty = threadIdx.x / kDnTile;
    const int px = blockIdx.x * kDnTile + tx, py = blockIdx.y * kDnTile + ty;
    if (px >= a.W || py >= a.H) return;
    const int64_t p = (int64_t)py * a.W + px;
    const int lx = tx + R, ly = ty + R;
    const float4 cc = lc[ly * span + lx], cn = ln[ly * span + lx];
    if (cn.w == 0.0f) {  // invalid: unchanged
        a.out[3 * p] = a.rgb[3 * p]; a.out[3 * p + 1] = a.rgb[3 * p + 1]; a.out[3 * p + 2] = a.rgb[3 * p + 2];
        return;
    }
    // depth gradient (R >= 1, so the four neighbours are staged)
    auto grad = [&](int ox, int oy) {
        const float4 pc = lc[(ly + oy) * span + lx + ox], mc = lc[(ly - oy) * span + lx - ox];
        const bool hp = ln[(ly + oy) * span + lx + ox].w != 0.0f, hm = ln[(ly - oy) * span + lx - ox].w != 0.0f;
        if (hp && hm) return (pc.w - mc.w) * 0.5f;
        if (hp) return pc.w - cc.w;
        if (hm) return cc.w - mc.w;
        return 0.0f;
    };
    const float gx = grad(1, 0), gy = grad(0, 1);
    const float inv2s2 = 1.0f / (2.0f * a.sigma_s * a.sigma_s);
    float sr = 0.0f, sg = 0.0f, sb = 0.0f, sw = 0.0f;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            const float4 qn = ln[(ly + dy) * span + lx + dx];
            if (qn.w == 0.0f) continue;
            const float4 qc = lc[(ly + dy) * span + lx + dx];
            const float ws = expf(-(float)(dx * dx + dy * dy) * inv2s2);
            const float wd = expf(-fabsf(cc.w - qc.w) / (a.sigma_d * fabsf(gx * (float)dx + gy * (float)dy) + a.eps_d));
            const float c = fmaxf(0.0f, cn.x * qn.x + cn.y * qn.y + cn.z * qn.z);
            const float B = ws * wd * powf(c, a.sigma_n);
            sr += B * qc.x; sg += B * qc.y; sb += B * qc.z; sw += B;
        }
    const float inv = sw > 0.0f ? 1.0f / sw : 1.0f;
    a.out[3 * p] = sr * inv; a.out[3 * p + 1] = sg * inv; a.out[3 * p + 2] = sb * inv;
}

hipError_t launch_denoise(const DenoiseArgs &a, hipStream_t st)
{
    if (a.H <= 0 || a.W <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.W + kDnTile - 1) / kDnTile), (unsigned)((a.H + kDnTile - 1) / kDnTile));
    hipLaunchKernelGGL(k_denoise, grid, dim3(kDnTile * kDnTile), 0, st, a);
    return hipGetLastError();
}

}  // namespace grt
