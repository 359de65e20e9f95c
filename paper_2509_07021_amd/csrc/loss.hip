// loss.hip -- the training-step pieces around the renderer, gfx950: the 3DGS photometric loss
// L = (1 - lambda) L1 + lambda (1 - SSIM) with its gradient, and an Adam step on parameter planes
// stored in FP32, FP16 or BF16 (the paper trains with 3DGS's loss, hyperparameters and optimiser;
// Appendix, experimental details).
//
// SSIM uses an 11x11 Gaussian window (sigma 1.5, separable, zero padding) and C1 = 0.01^2,
// C2 = 0.03^2. Writing S = a1 a2 / (b1 b2) with a1 = 2 mx my + C1, a2 = 2 sxy + C2,
// b1 = mx^2 + my^2 + C1, b2 = sxx + syy + C2, and the windowed raw moments (mx, Exx, Exy) as the
// variables, the derivative of S at pixel q with respect to x at pixel p is
//   G(p - q) (dS/dmx(q) + 2 x_p dS/dExx(q) + y_p dS/dExy(q)),
//   dS/dmx = (2 my (a2 - a1) - 2 mx S (b2 - b1)) / (b1 b2), dS/dExx = -S / b2, dS/dExy = 2 a1 / (b1 b2),
// so the gradient is a second windowed pass over those three maps. Both passes stage a tile and its
// 5-pixel halo in LDS and apply the window as a row pass then a column pass. The moments cancel
// (Exx - mx^2 against C2 = 9e-4), so all SSIM arithmetic is FP64; the planes are FP32. The loss sums
// go through per-workgroup partials reduced in a fixed order, so the loss is deterministic.
#include "megs_internal.hpp"

namespace megs {
namespace {

constexpr int kT = 16;              // output tile edge
constexpr int kR = 5;               // window radius
constexpr int kP = kT + 2 * kR;     // staged patch edge
constexpr double kC1 = 0.01 * 0.01, kC2 = 0.03 * 0.03;

__global__ __launch_bounds__(256) void k_ssim_fwd(LossView v, const float* __restrict__ x, const float* __restrict__ y,
                                                  double* __restrict__ maps, double* __restrict__ partial,
                                                  Window11 g) {
    __shared__ float sx[kP][kP], sy[kP][kP];
    __shared__ double hrow[kP][kT][5];
    __shared__ double red[2][256];
    const int tx = threadIdx.x % kT, ty = threadIdx.x / kT;
    const int tiles_x = (v.width + kT - 1) / kT;
    const int c = blockIdx.y;
    const int x0 = (blockIdx.x % tiles_x) * kT, y0 = (blockIdx.x / tiles_x) * kT;
    const int64_t plane = (int64_t)v.width * v.height;
    const float* xc = x + v.pix_off * 3 + c * plane;
    const float* yc = y + v.pix_off * 3 + c * plane;
    for (int i = threadIdx.x; i < kP * kP; i += 256) {
        const int r = i / kP, q = i % kP;
        const int gy = y0 - kR + r, gx = x0 - kR + q;
        const bool in = gx >= 0 && gy >= 0 && gx < v.width && gy < v.height;
        sx[r][q] = in ? xc[(int64_t)gy * v.width + gx] : 0.f;
        sy[r][q] = in ? yc[(int64_t)gy * v.width + gx] : 0.f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kP * kT; i += 256) {
        const int r = i / kT, q = i % kT;
        double s[5] = {0, 0, 0, 0, 0};
        for (int k = 0; k < 11; ++k) {
            const double a = sx[r][q + k], b = sy[r][q + k], w = g.w[k];
            s[0] += w * a; s[1] += w * b; s[2] += w * a * a; s[3] += w * b * b; s[4] += w * a * b;
        }
        for (int m = 0; m < 5; ++m) hrow[r][q][m] = s[m];
    }
    __syncthreads();
    double mo[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < 11; ++k)
        for (int m = 0; m < 5; ++m) mo[m] += g.w[k] * hrow[ty + k][tx][m];
    const int px = x0 + tx, py = y0 + ty;
    double ssim = 0.0, l1 = 0.0;
    if (px < v.width && py < v.height) {
        const double mx = mo[0], my = mo[1];
        const double a1 = 2.0 * mx * my + kC1, a2 = 2.0 * (mo[4] - mx * my) + kC2;
        const double b1 = mx * mx + my * my + kC1, b2 = (mo[2] - mx * mx) + (mo[3] - my * my) + kC2;
        const double den = b1 * b2;
        const double S = a1 * a2 / den;
        ssim = S;
        l1 = fabs((double)sx[ty + kR][tx + kR] - (double)sy[ty + kR][tx + kR]);
        const int64_t p = (int64_t)py * v.width + px;
        double* mc = maps + (v.pix_off * 3 + c * plane) * 3;
        mc[p] = (2.0 * my * (a2 - a1) - 2.0 * mx * S * (b2 - b1)) / den;
        mc[plane + p] = -S / b2;
        mc[2 * plane + p] = 2.0 * a1 / den;
    }
    red[0][threadIdx.x] = ssim;
    red[1][threadIdx.x] = l1;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t b = v.part_off + (int64_t)c * gridDim.x + blockIdx.x;
        partial[2 * b] = red[0][0];
        partial[2 * b + 1] = red[1][0];
    }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(LossView v, const float* __restrict__ x, const float* __restrict__ y,
                                                  const double* __restrict__ maps, float* __restrict__ dl, Window11 g,
                                                  double lam) {
    __shared__ double sm[3][kP][kP];
    __shared__ double hrow[kP][kT][3];
    const int tx = threadIdx.x % kT, ty = threadIdx.x / kT;
    const int tiles_x = (v.width + kT - 1) / kT;
    const int c = blockIdx.y;
    const int x0 = (blockIdx.x % tiles_x) * kT, y0 = (blockIdx.x / tiles_x) * kT;
    const int64_t plane = (int64_t)v.width * v.height;
    const double* mc = maps + (v.pix_off * 3 + c * plane) * 3;
    for (int i = threadIdx.x; i < kP * kP; i += 256) {
        const int r = i / kP, q = i % kP;
        const int gy = y0 - kR + r, gx = x0 - kR + q;
        const bool in = gx >= 0 && gy >= 0 && gx < v.width && gy < v.height;
        const int64_t p = (int64_t)gy * v.width + gx;
        for (int m = 0; m < 3; ++m) sm[m][r][q] = in ? mc[m * plane + p] : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kP * kT; i += 256) {
        const int r = i / kT, q = i % kT;
        double s[3] = {0, 0, 0};
        for (int k = 0; k < 11; ++k)
            for (int m = 0; m < 3; ++m) s[m] += g.w[k] * sm[m][r][q + k];
        for (int m = 0; m < 3; ++m) hrow[r][q][m] = s[m];
    }
    __syncthreads();
    const int px = x0 + tx, py = y0 + ty;
    if (px >= v.width || py >= v.height) return;
    double b[3] = {0, 0, 0};
    for (int k = 0; k < 11; ++k)
        for (int m = 0; m < 3; ++m) b[m] += g.w[k] * hrow[ty + k][tx][m];
    const int64_t p = (int64_t)py * v.width + px;
    const int64_t off = v.pix_off * 3 + c * plane + p;
    const double xv = x[off], yv = y[off];
    const double n = 3.0 * (double)plane;
    const double sgn = xv > yv ? 1.0 : (xv < yv ? -1.0 : 0.0);
    const double dssim = b[0] + 2.0 * xv * b[1] + yv * b[2];
    dl[off] = (float)((1.0 - lam) * sgn / n - lam * dssim / n);
}

// One workgroup per view: the view's loss term from its partial sums, in a fixed order.
__global__ __launch_bounds__(256) void k_loss_views(const double* __restrict__ partial, const LossViews vs,
                                                    double lam, double* __restrict__ terms) {
    __shared__ double red[2][256];
    const LossView& v = vs.v[blockIdx.x];
    double s = 0.0, l = 0.0;
    for (int64_t b = threadIdx.x; b < v.n_part; b += 256) {
        s += partial[2 * (v.part_off + b)];
        l += partial[2 * (v.part_off + b) + 1];
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = l;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            red[0][threadIdx.x] += red[0][threadIdx.x + k];
            red[1][threadIdx.x] += red[1][threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = 3.0 * (double)v.width * v.height;
        terms[blockIdx.x] = (1.0 - lam) * red[1][0] / n + lam * (1.0 - red[0][0] / n);
    }
}

__global__ void k_loss_total(const double* __restrict__ terms, int nv, double* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nv; ++i) s += terms[i];
    loss[0] = s;
}

// Adam (Kingma and Ba) with bias correction, FP32 arithmetic; the parameter is read from and
// written back to its storage dtype (round to nearest even).
__global__ __launch_bounds__(256) void k_adam(int64_t count, void* __restrict__ param, int dt,
                                              const float* __restrict__ grad, float* __restrict__ m,
                                              float* __restrict__ v, float lr, float b1, float b2, float eps,
                                              float bc1, float bc2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float mi = __fmaf_rn(b1, m[i], (1.0f - b1) * gi);
        const float vi = __fmaf_rn(b2, v[i], (1.0f - b2) * gi * gi);
        m[i] = mi;
        v[i] = vi;
        const float upd = lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
        store_elem(param, dt, i, load_elem(param, dt, i) - upd);
    }
}

}  // namespace

hipError_t launch_loss(const LossViews& vs, int nv, const float* x, const float* y, double* maps, double* partial,
                       double* terms, double* loss, float* dl, const Window11& g, double lam, hipStream_t stream) {
    for (int i = 0; i < nv; ++i) {
        const LossView& v = vs.v[i];
        const int tiles = ((v.width + kT - 1) / kT) * ((v.height + kT - 1) / kT);
        hipLaunchKernelGGL(k_ssim_fwd, dim3(tiles, 3), dim3(256), 0, stream, v, x, y, maps, partial, g);
    }
    hipLaunchKernelGGL(k_loss_views, dim3(nv), dim3(256), 0, stream, partial, vs, lam, terms);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, stream, terms, nv, loss);
    if (dl) {
        for (int i = 0; i < nv; ++i) {
            const LossView& v = vs.v[i];
            const int tiles = ((v.width + kT - 1) / kT) * ((v.height + kT - 1) / kT);
            hipLaunchKernelGGL(k_ssim_bwd, dim3(tiles, 3), dim3(256), 0, stream, v, x, y, maps, dl, g, lam);
        }
    }
    return hipGetLastError();
}

int64_t loss_partials(int width, int height) {
    return 3ll * ((width + kT - 1) / kT) * ((height + kT - 1) / kT);
}

hipError_t launch_adam(int64_t count, void* param, int dt, const float* grad, float* m, float* v, float lr, float b1,
                       float b2, float eps, int step, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const float bc1 = (float)(1.0 - pow((double)b1, step)), bc2 = (float)(1.0 - pow((double)b2, step));
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, stream, count, param, dt, grad, m, v, lr, b1, b2,
                       eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace megs
