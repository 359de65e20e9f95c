// project.hip -- EWA projection with Spherical-Gaussian colour (forward) and its chain rule
// back to the raw parameters (backward), gfx950.
//
// One thread per Gaussian loops over all views, so the parameter planes are streamed from HBM
// once per launch (coalesced SoA loads, widened from FP16/BF16 in registers) and the records of
// every view are written. View-independent values (activations, 3D covariance, unit lobe axes,
// base colour) are formed once per Gaussian. The camera-space position, the pixel mean and the
// tile count (the row-interval test of the key emission) are computed in FP64, everything else in
// FP32. The kernels are bound by the latency of their dependent arithmetic at the occupancy their
// registers allow (four and three waves per SIMD).
//
// Colour: c(d) = c0 + sum_k m_k a_k exp(lambda_k (mu_k . d - 1)) (SG lobe and colour equations,
// Sec. 3.2), with lambda (mu . d - 1) evaluated as -lambda |mu - d|^2 / 2 for unit mu and d, which
// is the same quantity without the cancellation of mu . d - 1 near the lobe axis.
#include "megs_internal.hpp"

namespace megs {
namespace {

struct Geo {
    float s[3];
    float qh[4];
    float Rq[9];
    float S3[6];  // xx, xy, xz, yy, yz, zz
    float o, mp, o_eff;
    float qnorm;
    bool ok;
};

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + __expf(-x)); }

template <int K>
struct Lobes {
    float mu[K > 0 ? K : 1][3];  // unit lobe axes mu / |mu| (view-independent, formed once)
    float ia[K > 0 ? K : 1];     // 1 / |mu| of the raw axes
    float lam[K > 0 ? K : 1];
    float amp[K > 0 ? K : 1][3];
    float m[K > 0 ? K : 1];
};

__device__ __forceinline__ void rot_from_quat(const float q[4], float R[9]) {
    float w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

// View-independent part: activations and the 3D covariance.
__device__ __forceinline__ void load_geo(const SceneDev& sc, int64_t i, float pos[3], Geo& g) {
    const int64_t n = sc.n;
    for (int j = 0; j < 3; ++j) pos[j] = load_elem(sc.pos, sc.dt_geom, j * n + i);
    for (int j = 0; j < 3; ++j) g.s[j] = __expf(load_elem(sc.logscale, sc.dt_geom, j * n + i));
    float q[4];
    for (int j = 0; j < 4; ++j) q[j] = load_elem(sc.quat, sc.dt_geom, j * n + i);
    float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    g.ok = (qq > 0.0f) && isfinite(qq);
    g.qnorm = sqrtf(qq);
    float inv = 1.0f / g.qnorm;
    for (int j = 0; j < 4; ++j) g.qh[j] = q[j] * inv;
    rot_from_quat(g.qh, g.Rq);
    float M[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = g.Rq[3 * r + c] * g.s[c];
    g.S3[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    g.S3[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    g.S3[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    g.S3[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    g.S3[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    g.S3[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
    g.o = sigmoidf(load_elem(sc.op_logit, sc.dt_geom, i));
    g.mp = sc.pmask_logit ? sigmoidf(load_elem(sc.pmask_logit, sc.dt_geom, i)) : 1.0f;
    g.o_eff = g.o * g.mp;
}

// Lobe slots at or past the Gaussian's count get zero mask and amplitude, so they add exactly +0.
template <int K, bool RAGGED>
__device__ __forceinline__ bool load_lobes(const SceneDev& sc, const LobeRef<RAGGED>& r, Lobes<K>& L) {
    bool ok = true;
#pragma unroll
    for (int l = 0; l < K; ++l) {
        if (RAGGED && l >= r.cnt) {
            L.mu[l][0] = 1.0f; L.mu[l][1] = 0.0f; L.mu[l][2] = 0.0f;
            L.ia[l] = 1.0f;
            L.lam[l] = 0.0f; L.m[l] = 0.0f;
            L.amp[l][0] = L.amp[l][1] = L.amp[l][2] = 0.0f;
            continue;
        }
        float a0 = load_elem(sc.axis, sc.dt_color, r.at3(l, 0));
        float a1 = load_elem(sc.axis, sc.dt_color, r.at3(l, 1));
        float a2 = load_elem(sc.axis, sc.dt_color, r.at3(l, 2));
        float al2 = a0 * a0 + a1 * a1 + a2 * a2;
        const float ia = rsqrtf(al2);
        L.ia[l] = ia;
        L.mu[l][0] = a0 * ia; L.mu[l][1] = a1 * ia; L.mu[l][2] = a2 * ia;
        ok = ok && (al2 > 0.0f) && isfinite(al2);
        L.lam[l] = load_elem(sc.sharp, sc.dt_color, r.at1(l));
#pragma unroll
        for (int c = 0; c < 3; ++c) L.amp[l][c] = load_elem(sc.amp, sc.dt_amp, r.at3(l, c));
        L.m[l] = sc.lmask_logit ? sigmoidf(load_elem(sc.lmask_logit, sc.dt_color, r.at1(l))) : 1.0f;
    }
    return ok;
}

// Per-view projection intermediates (shared by forward and backward so both take the same
// culling decisions and see the same values).
struct ViewProj {
    bool ok;
    double tx, ty, tz, u, v;
    float txf, tyf, tzf, xi, eta;
    bool xclamp, yclamp;
    float T0[3], T1[3];
    float A0, B0, C0, det0, det;
    float conic[3];
    int32_t radius;
};

__device__ __forceinline__ void project_view(const Geo& g, const float pos[3], const ViewInfo& vw, ViewProj& p) {
    p.ok = g.ok;
    const double px = pos[0], py = pos[1], pz = pos[2];
    p.tx = fma((double)vw.R[0], px, fma((double)vw.R[1], py, fma((double)vw.R[2], pz, (double)vw.t[0])));
    p.ty = fma((double)vw.R[3], px, fma((double)vw.R[4], py, fma((double)vw.R[5], pz, (double)vw.t[1])));
    p.tz = fma((double)vw.R[6], px, fma((double)vw.R[7], py, fma((double)vw.R[8], pz, (double)vw.t[2])));
    if (!(p.tz > (double)vw.znear)) p.ok = false;
    if (!(g.o_eff >= kAlphaMin)) p.ok = false;
    const double rz = 1.0 / p.tz;
    p.u = fma((double)vw.fx * p.tx, rz, (double)vw.cx);
    p.v = fma((double)vw.fy * p.ty, rz, (double)vw.cy);
    p.txf = (float)p.tx; p.tyf = (float)p.ty; p.tzf = (float)p.tz;
    float rx = (float)(p.tx * rz), ry = (float)(p.ty * rz);
    p.xclamp = rx < -vw.limx || rx > vw.limx;
    p.yclamp = ry < -vw.limy || ry > vw.limy;
    p.xi = fminf(fmaxf(rx, -vw.limx), vw.limx);
    p.eta = fminf(fmaxf(ry, -vw.limy), vw.limy);
    const float irz = 1.0f / p.tzf;
    const float J00 = vw.fx * irz, J02 = -vw.fx * p.xi * irz;
    const float J11 = vw.fy * irz, J12 = -vw.fy * p.eta * irz;
    // T = J W: row 0 = J00 W0 + J02 W2, row 1 = J11 W1 + J12 W2
    for (int c = 0; c < 3; ++c) {
        p.T0[c] = J00 * vw.R[c] + J02 * vw.R[6 + c];
        p.T1[c] = J11 * vw.R[3 + c] + J12 * vw.R[6 + c];
    }
    // S3 * T0 and S3 * T1
    const float* S = g.S3;
    float s0[3] = {S[0] * p.T0[0] + S[1] * p.T0[1] + S[2] * p.T0[2],
                   S[1] * p.T0[0] + S[3] * p.T0[1] + S[4] * p.T0[2],
                   S[2] * p.T0[0] + S[4] * p.T0[1] + S[5] * p.T0[2]};
    float s1[3] = {S[0] * p.T1[0] + S[1] * p.T1[1] + S[2] * p.T1[2],
                   S[1] * p.T1[0] + S[3] * p.T1[1] + S[4] * p.T1[2],
                   S[2] * p.T1[0] + S[4] * p.T1[1] + S[5] * p.T1[2]};
    p.A0 = p.T0[0] * s0[0] + p.T0[1] * s0[1] + p.T0[2] * s0[2];
    p.B0 = p.T0[0] * s1[0] + p.T0[1] * s1[1] + p.T0[2] * s1[2];
    p.C0 = p.T1[0] * s1[0] + p.T1[1] * s1[1] + p.T1[2] * s1[2];
    p.det0 = p.A0 * p.C0 - p.B0 * p.B0;
    p.det = fmaxf(p.det0, 0.0f) + kDilation * (p.A0 + p.C0) + kDilation * kDilation;
    const float A = p.A0 + kDilation, C = p.C0 + kDilation;
    const float idet = 1.0f / p.det;
    p.conic[0] = C * idet;
    p.conic[1] = -p.B0 * idet;
    p.conic[2] = A * idet;
    const float mid = 0.5f * (A + C);
    const float lmax = mid + sqrtf(fmaxf(mid * mid - p.det, 0.0f));
    const float rho = sqrtf(2.0f * __logf(255.0f * g.o_eff) * lmax);
    const float r = ceilf(rho);
    if (!(isfinite(p.u) && isfinite(p.v) && isfinite(r)) || fabs(p.u) > kMaxCoord || fabs(p.v) > kMaxCoord ||
        r > (float)kMaxCoord)
        p.ok = false;
    p.radius = p.ok ? (int32_t)r : -1;
}

// d = (mu - campos) / |mu - campos|, the viewing direction (from the camera to the Gaussian).
__device__ __forceinline__ void view_dir(const float pos[3], const ViewInfo& vw, float d[3], float& dlen) {
    float dv[3] = {pos[0] - vw.campos[0], pos[1] - vw.campos[1], pos[2] - vw.campos[2]};
    dlen = sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    const float il = 1.0f / dlen;
    d[0] = dv[0] * il; d[1] = dv[1] * il; d[2] = dv[2] * il;
}

// The base colour c0 of Gaussian i (view-independent; read once, before the view loop).
__device__ __forceinline__ void load_base(const SceneDev& sc, int64_t i, float base[3]) {
    for (int c = 0; c < 3; ++c) base[c] = load_elem(sc.base, sc.dt_color, c * sc.n + i);
}

// The SG colour at d; returns false if not finite.
template <int K>
__device__ __forceinline__ bool sg_colour(const float base[3], const float pos[3], const ViewInfo& vw,
                                          const Lobes<K>& L, float d[3], float& dlen, float rgb[3], float e[K > 0 ? K : 1],
                                          float muh[K > 0 ? K : 1][3], float dd2[K > 0 ? K : 1]) {
    view_dir(pos, vw, d, dlen);
    for (int c = 0; c < 3; ++c) rgb[c] = base[c];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        float df2 = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            muh[l][c] = L.mu[l][c];
            const float df = muh[l][c] - d[c];
            df2 += df * df;
        }
        dd2[l] = df2;
        e[l] = __expf(-0.5f * L.lam[l] * df2);
        const float w = L.m[l] * e[l];
#pragma unroll
        for (int c = 0; c < 3; ++c) rgb[c] += w * L.amp[l][c];
    }
    return isfinite(rgb[0]) && isfinite(rgb[1]) && isfinite(rgb[2]);
}

// ---- spherical-harmonic colour (3DGS's colour model, for the same-renderer comparison) ----
// Real spherical harmonics of degree <= D at a unit direction (x, y, z), orthonormal over the
// sphere, in the sign convention of the 3DGS rasteriser: Y_0 = 1 / (2 sqrt(pi)); degree 1:
// sqrt(3 / (4 pi)) (-y, z, -x); degree 2 and 3: the Cartesian polynomials below with their
// normalisations (sqrt(15 / pi) / 2, sqrt(5 / pi) / 4, sqrt(15 / pi) / 4; sqrt(35 / (2 pi)) / 4,
// sqrt(105 / pi) / 2, sqrt(21 / (2 pi)) / 4, sqrt(7 / pi) / 4, sqrt(105 / pi) / 4).
constexpr float kSh0 = 0.28209479177387814f;
constexpr float kSh1 = 0.48860251190291992f;
constexpr float kSh2a = 1.0925484305920792f, kSh2b = 0.31539156525252005f, kSh2c = 0.54627421529603959f;
constexpr float kSh3a = 0.59004358992664352f, kSh3b = 2.8906114426405538f, kSh3c = 0.45704579946446572f;
constexpr float kSh3d = 0.37317633259011540f, kSh3e = 1.4453057213202769f;

// Basis values Y[m] and, when G, their partial derivatives dY[m][0..2] in x, y, z (polynomials
// extended off the sphere; callers project onto the tangent plane).
template <int D, bool G>
__device__ __forceinline__ void sh_basis(const float d[3], float Y[16], float dY[16][3]) {
    const float x = d[0], y = d[1], z = d[2];
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = kSh0;
    if (G) dY[0][0] = dY[0][1] = dY[0][2] = 0.f;
    if (D >= 1) {
        Y[1] = -kSh1 * y; Y[2] = kSh1 * z; Y[3] = -kSh1 * x;
        if (G) {
            dY[1][0] = 0.f; dY[1][1] = -kSh1; dY[1][2] = 0.f;
            dY[2][0] = 0.f; dY[2][1] = 0.f; dY[2][2] = kSh1;
            dY[3][0] = -kSh1; dY[3][1] = 0.f; dY[3][2] = 0.f;
        }
    }
    if (D >= 2) {
        Y[4] = kSh2a * x * y;
        Y[5] = -kSh2a * y * z;
        Y[6] = kSh2b * (2.f * zz - xx - yy);
        Y[7] = -kSh2a * x * z;
        Y[8] = kSh2c * (xx - yy);
        if (G) {
            dY[4][0] = kSh2a * y; dY[4][1] = kSh2a * x; dY[4][2] = 0.f;
            dY[5][0] = 0.f; dY[5][1] = -kSh2a * z; dY[5][2] = -kSh2a * y;
            dY[6][0] = -2.f * kSh2b * x; dY[6][1] = -2.f * kSh2b * y; dY[6][2] = 4.f * kSh2b * z;
            dY[7][0] = -kSh2a * z; dY[7][1] = 0.f; dY[7][2] = -kSh2a * x;
            dY[8][0] = 2.f * kSh2c * x; dY[8][1] = -2.f * kSh2c * y; dY[8][2] = 0.f;
        }
    }
    if (D >= 3) {
        const float q = 4.f * zz - xx - yy;
        Y[9] = -kSh3a * y * (3.f * xx - yy);
        Y[10] = kSh3b * x * y * z;
        Y[11] = -kSh3c * y * q;
        Y[12] = kSh3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
        Y[13] = -kSh3c * x * q;
        Y[14] = kSh3e * z * (xx - yy);
        Y[15] = -kSh3a * x * (xx - 3.f * yy);
        if (G) {
            dY[9][0] = -6.f * kSh3a * x * y; dY[9][1] = -3.f * kSh3a * (xx - yy); dY[9][2] = 0.f;
            dY[10][0] = kSh3b * y * z; dY[10][1] = kSh3b * x * z; dY[10][2] = kSh3b * x * y;
            dY[11][0] = 2.f * kSh3c * x * y; dY[11][1] = -kSh3c * (q - 2.f * yy); dY[11][2] = -8.f * kSh3c * y * z;
            dY[12][0] = -6.f * kSh3d * x * z; dY[12][1] = -6.f * kSh3d * y * z;
            dY[12][2] = kSh3d * (6.f * zz - 3.f * xx - 3.f * yy);
            dY[13][0] = -kSh3c * (q - 2.f * xx); dY[13][1] = 2.f * kSh3c * x * y; dY[13][2] = -8.f * kSh3c * x * z;
            dY[14][0] = 2.f * kSh3e * x * z; dY[14][1] = -2.f * kSh3e * y * z; dY[14][2] = kSh3e * (xx - yy);
            dY[15][0] = -3.f * kSh3a * (xx - yy); dY[15][1] = 6.f * kSh3a * x * y; dY[15][2] = 0.f;
        }
    }
}

// colour = max(0, sum_m Y_m(d) sh[m] + 1/2) per channel; clamped[c] records the clamp.
template <int D>
__device__ __forceinline__ bool sh_colour(const SceneDev& sc, int64_t i, const float pos[3], const ViewInfo& vw,
                                          float d[3], float& dlen, float rgb[3], bool clamped[3]) {
    constexpr int M = (D + 1) * (D + 1);
    const int64_t n = sc.n;
    view_dir(pos, vw, d, dlen);
    float Y[16], dY[16][3];
    sh_basis<D, false>(d, Y, dY);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float acc = 0.5f;
#pragma unroll
        for (int m = 0; m < M; ++m) acc = __fmaf_rn(Y[m], load_elem(sc.sh, sc.dt_color, ((int64_t)m * 3 + c) * n + i), acc);
        clamped[c] = acc < 0.0f;
        rgb[c] = clamped[c] ? 0.0f : acc;
    }
    return isfinite(rgb[0]) && isfinite(rgb[1]) && isfinite(rgb[2]);
}

// Ellipse level that bounds every pixel with alpha >= 1/255: q <= 2 ln(255 o), widened by 0.2% (and
// 1e-4 absolute) so that FP32 rounding in the blend never reaches past a culled tile.
__device__ __forceinline__ float cutoff_of(float o_eff) {
    return 2.004f * __logf(255.0f * o_eff) + 1e-4f;
}

template <int K, bool RAGGED, int SHD>
__global__ __launch_bounds__(256) void k_project(SceneDev sc, const ViewInfo* __restrict__ views, int nv, int tile,
                                                 Records rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.n) return;
    float pos[3];
    Geo g;
    load_geo(sc, i, pos, g);
    Lobes<K> L;
    LobeRef<RAGGED> lr;
    const bool lobes_ok = lobe_ref<RAGGED>(sc, i, K, lr) && load_lobes<K, RAGGED>(sc, lr, L);
    float base[3] = {0.f, 0.f, 0.f};
    if constexpr (SHD < 0) load_base(sc, i, base);
    for (int v = 0; v < nv; ++v) {
        const ViewInfo& vw = views[v];
        const int64_t r = (int64_t)v * sc.n + i;
        ViewProj p;
        project_view(g, pos, vw, p);
        float d[3], dlen, rgb[3], e[K > 0 ? K : 1], muh[K > 0 ? K : 1][3], dd2[K > 0 ? K : 1];
        bool ok = p.ok && lobes_ok;
        if (ok) {
            if constexpr (SHD >= 0) {
                bool clamped[3];
                ok = sh_colour<SHD>(sc, i, pos, vw, d, dlen, rgb, clamped);
            } else {
                ok = sg_colour<K>(base, pos, vw, L, d, dlen, rgb, e, muh, dd2);
            }
        }
        uint32_t nt = 0;
        if (ok) {
            int x0, x1, y0, y1;
            const float cut = cutoff_of(g.o_eff);
            if (tile_rect(p.u, p.v, p.radius, vw, tile, x0, x1, y0, y1)) {
                EllipseRows er;
                ellipse_rows(p.u, p.v, p.conic[0], p.conic[1], p.conic[2], cut, er);
                for (int ty = y0; ty <= y1; ++ty) {
                    int lo, hi;
                    if (row_span(er, vw.width, vw.height, tile, ty, x0, x1, lo, hi)) nt += (uint32_t)(hi - lo + 1);
                }
            }
            if (rec.mean) {  // per-field planes, on request only
                rec.mean[r] = make_double2(p.u, p.v);
                rec.conic_o[r] = make_float4(p.conic[0], p.conic[1], p.conic[2], g.o_eff);
                rec.rgbd[r] = make_float4(rgb[0], rgb[1], rgb[2], p.tzf);
                rec.radius[r] = p.radius;
                rec.cutoff[r] = cut;
            }
        } else if (rec.mean) {
            rec.mean[r] = make_double2(0.0, 0.0);
            rec.conic_o[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            rec.rgbd[r] = make_float4(0.f, 0.f, 0.f, 0.f);
            rec.radius[r] = -1;
            rec.cutoff[r] = 0.f;
        }
        rec.ntiles[r] = nt;
        {
            // packed copy; the half-extents of the cutoff ellipse {q <= k} are sqrt(k S_xx) and
            // sqrt(k S_yy) with S_xx = c / (a c - b^2), S_yy = a / (a c - b^2), the FP32 conic's
            // determinant taken in FP64 (products of FP32 values are exact there, so thin ellipses
            // keep their extent) and rounded once to FP32; the rest in FP32 with the hardware
            // reciprocal and square root (about 1 ulp each), far inside the widening by 1e-3
            // relative and 1e-2 px: every pixel with alpha >= 1/255 lies inside the box
            float rx = 0.f, ry = 0.f;
            if (ok) {
                const double detd = (double)p.conic[0] * p.conic[2] - (double)p.conic[1] * p.conic[1];
                const float kd = cutoff_of(g.o_eff) * __builtin_amdgcn_rcpf((float)detd);
                rx = detd > 0.0 ? __builtin_amdgcn_sqrtf(kd * p.conic[2]) * 1.001f + 0.01f : 1e30f;
                ry = detd > 0.0 ? __builtin_amdgcn_sqrtf(kd * p.conic[0]) * 1.001f + 0.01f : 1e30f;
            }
            PackedRec pr;
            pr.mean = ok ? make_double2(p.u, p.v) : make_double2(0.0, 0.0);
            pr.conic_o = ok ? make_float4(p.conic[0], p.conic[1], p.conic[2], g.o_eff) : make_float4(0.f, 0.f, 0.f, 0.f);
            pr.rgbk = ok ? make_float4(rgb[0], rgb[1], rgb[2], cutoff_of(g.o_eff)) : make_float4(0.f, 0.f, 0.f, 0.f);
            pr.radius = ok ? p.radius : -1;
            pr.ntiles = nt;
            pr.rx = rx;
            pr.ry = ry;
            float4* dst = reinterpret_cast<float4*>(rec.packed + r);
            const float4* src = reinterpret_cast<const float4*>(&pr);
            dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2]; dst[3] = src[3];
        }
        rec.dkey[r] = nt ? __float_as_uint(p.tzf) : 0xffffffffu;
        if (rec.order0) {
            const uint32_t cap = (1u << (32 - rec.order_idb)) - 1u;
            rec.order0[r] = (min(nt, cap) << rec.order_idb) | (uint32_t)r;
        }
    }
}

// ----------------------------------------------------------------- backward ----

__device__ __forceinline__ void quat_grad(const float q[4], const float gR[9], float gq[4]) {
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    // d R / d (w, x, y, z) contracted with gR, for R of a unit quaternion (textbook form)
    gq[0] = 2.f * (z * (gR[3] - gR[1]) + y * (gR[2] - gR[6]) + x * (gR[7] - gR[5]));
    gq[1] = 2.f * (y * (gR[1] + gR[3]) + z * (gR[2] + gR[6]) + w * (gR[7] - gR[5])) - 4.f * x * (gR[4] + gR[8]);
    gq[2] = 2.f * (x * (gR[1] + gR[3]) + w * (gR[2] - gR[6]) + z * (gR[5] + gR[7])) - 4.f * y * (gR[0] + gR[8]);
    gq[3] = 2.f * (w * (gR[3] - gR[1]) + x * (gR[2] + gR[6]) + y * (gR[5] + gR[7])) - 4.f * z * (gR[0] + gR[4]);
}

template <int K, bool RAGGED, int SHD>
__device__ __forceinline__ void project_bwd_one(const SceneDev& sc, const ViewInfo* __restrict__ views, int nv,
                                                const float* __restrict__ grad2d, const GradDev& G) {
    constexpr int SHM = SHD >= 0 ? (SHD + 1) * (SHD + 1) : 1;
    float gsh[SHM][3];
#pragma unroll
    for (int m = 0; m < SHM; ++m) gsh[m][0] = gsh[m][1] = gsh[m][2] = 0.f;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.n) return;
    const int64_t n = sc.n;
    float pos[3];
    Geo g;
    load_geo(sc, i, pos, g);
    Lobes<K> L;
    LobeRef<RAGGED> lr;
    const bool lobes_ok = lobe_ref<RAGGED>(sc, i, K, lr) && load_lobes<K, RAGGED>(sc, lr, L);
    float base[3] = {0.f, 0.f, 0.f};
    if constexpr (SHD < 0) load_base(sc, i, base);

    float gpos[3] = {0.f, 0.f, 0.f}, gS3[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float gop = 0.f, gpm = 0.f, gbase[3] = {0.f, 0.f, 0.f};
    constexpr int KK = K > 0 ? K : 1;
    float gax[KK][3], glam[KK], gamp[KK][3], glm[KK];
#pragma unroll
    for (int l = 0; l < KK; ++l) {
        gax[l][0] = gax[l][1] = gax[l][2] = 0.f;
        glam[l] = 0.f; glm[l] = 0.f;
        gamp[l][0] = gamp[l][1] = gamp[l][2] = 0.f;
    }

    for (int v = 0; v < nv; ++v) {
        const ViewInfo& vw = views[v];
        const int64_t r = (int64_t)v * n + i;
        ViewProj p;
        project_view(g, pos, vw, p);
        float d[3], dlen, rgb[3], e[KK], muh[KK][3], dd2[KK];
        bool clamped[3] = {false, false, false};
        bool ok = p.ok && lobes_ok;
        if (ok) {
            if constexpr (SHD >= 0)
                ok = sh_colour<SHD>(sc, i, pos, vw, d, dlen, rgb, clamped);
            else
                ok = sg_colour<K>(base, pos, vw, L, d, dlen, rgb, e, muh, dd2);
        }
        if (!ok) continue;
        // The blend leaves, over the record's fragments, e = dL/do_eff per fragment (unclamped ones;
        // go below is their sum) and the moments sum e dx, e dy, e dx^2, e dx dy, e dy^2, (dx, dy)
        // the pixel offset from the mean. The exponent q = -(a dx^2 + 2 b dx dy + c dy^2) / 2 has
        // dL/dq = o_eff e, so the gradients of the pixel mean and of the conic (a, b, c) follow here,
        // once per record.
        const float* gr = grad2d + 9 * r;
        const float oe = g.o_eff;
        const float m0 = oe * gr[0], m1 = oe * gr[1];
        const float gu = p.conic[0] * m0 + p.conic[1] * m1;
        const float gv = p.conic[1] * m0 + p.conic[2] * m1;
        const float ga = -0.5f * oe * gr[2], gb = -oe * gr[3], gc = -0.5f * oe * gr[4], go = gr[5];
        const float gcol[3] = {gr[6], gr[7], gr[8]};

        // colour
        float gd[3] = {0.f, 0.f, 0.f};
        if constexpr (SHD >= 0) {
            float Y[16], dY[16][3];
            sh_basis<SHD, true>(d, Y, dY);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float gc = clamped[c] ? 0.f : gcol[c];
#pragma unroll
                for (int m = 0; m < SHM; ++m) {
                    gsh[m][c] = __fmaf_rn(Y[m], gc, gsh[m][c]);
                    const float w = gc * load_elem(sc.sh, sc.dt_color, ((int64_t)m * 3 + c) * n + i);
                    gd[0] = __fmaf_rn(w, dY[m][0], gd[0]);
                    gd[1] = __fmaf_rn(w, dY[m][1], gd[1]);
                    gd[2] = __fmaf_rn(w, dY[m][2], gd[2]);
                }
            }
        } else {
            for (int c = 0; c < 3; ++c) gbase[c] += gcol[c];
        }
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const float ip = L.amp[l][0] * gcol[0] + L.amp[l][1] * gcol[1] + L.amp[l][2] * gcol[2];
            const float w = L.m[l] * e[l];
            for (int c = 0; c < 3; ++c) gamp[l][c] += w * gcol[c];
            glam[l] += w * (-0.5f * dd2[l]) * ip;
            const float coef = w * L.lam[l] * ip;
            const float md = muh[l][0] * d[0] + muh[l][1] * d[1] + muh[l][2] * d[2];
            const float ial = L.ia[l];
            for (int c = 0; c < 3; ++c) {
                gax[l][c] += coef * (d[c] - muh[l][c] * md) * ial;
                gd[c] += coef * muh[l][c];
            }
            glm[l] += L.m[l] * (1.f - L.m[l]) * e[l] * ip;
        }
        {
            const float dg = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
            const float il = 1.0f / dlen;
            for (int c = 0; c < 3; ++c) gpos[c] += (gd[c] - d[c] * dg) * il;
        }
        // opacity and primitive mask
        gop += go * g.mp * g.o * (1.f - g.o);
        gpm += go * g.o * g.mp * (1.f - g.mp);

        // conic = (C, -B, A) / det, A = A0 + h, C = C0 + h
        const float A = p.A0 + kDilation, C = p.C0 + kDilation, B = p.B0;
        const float idet = 1.0f / p.det;
        const float gdet = -(ga * C - gb * B + gc * A) * idet * idet;
        float gA0 = gc * idet, gC0 = ga * idet, gB0 = -gb * idet;
        if (p.det0 > 0.f) {
            gA0 += gdet * C;
            gC0 += gdet * A;
            gB0 -= 2.f * B * gdet;
        } else {
            gA0 += gdet * kDilation;
            gC0 += gdet * kDilation;
        }
        // Sigma2 entries A0 = T0 S T0', B0 = T0 S T1', C0 = T1 S T1'
        const float* T0 = p.T0;
        const float* T1 = p.T1;
        gS3[0] += gA0 * T0[0] * T0[0] + gB0 * T0[0] * T1[0] + gC0 * T1[0] * T1[0];
        gS3[3] += gA0 * T0[1] * T0[1] + gB0 * T0[1] * T1[1] + gC0 * T1[1] * T1[1];
        gS3[5] += gA0 * T0[2] * T0[2] + gB0 * T0[2] * T1[2] + gC0 * T1[2] * T1[2];
        gS3[1] += 2.f * gA0 * T0[0] * T0[1] + gB0 * (T0[0] * T1[1] + T1[0] * T0[1]) + 2.f * gC0 * T1[0] * T1[1];
        gS3[2] += 2.f * gA0 * T0[0] * T0[2] + gB0 * (T0[0] * T1[2] + T1[0] * T0[2]) + 2.f * gC0 * T1[0] * T1[2];
        gS3[4] += 2.f * gA0 * T0[1] * T0[2] + gB0 * (T0[1] * T1[2] + T1[1] * T0[2]) + 2.f * gC0 * T1[1] * T1[2];
        // gradient w.r.t. T rows: dA0/dT0 = 2 S T0, dB0/dT0 = S T1, dB0/dT1 = S T0, dC0/dT1 = 2 S T1
        const float* S = g.S3;
        const float sT0[3] = {S[0] * T0[0] + S[1] * T0[1] + S[2] * T0[2], S[1] * T0[0] + S[3] * T0[1] + S[4] * T0[2],
                              S[2] * T0[0] + S[4] * T0[1] + S[5] * T0[2]};
        const float sT1[3] = {S[0] * T1[0] + S[1] * T1[1] + S[2] * T1[2], S[1] * T1[0] + S[3] * T1[1] + S[4] * T1[2],
                              S[2] * T1[0] + S[4] * T1[1] + S[5] * T1[2]};
        float gT0[3], gT1[3];
        for (int c = 0; c < 3; ++c) {
            gT0[c] = 2.f * gA0 * sT0[c] + gB0 * sT1[c];
            gT1[c] = 2.f * gC0 * sT1[c] + gB0 * sT0[c];
        }
        // T0 = J00 W0 + J02 W2, T1 = J11 W1 + J12 W2 (W rows of the camera rotation)
        const float* W = vw.R;
        const float gJ00 = gT0[0] * W[0] + gT0[1] * W[1] + gT0[2] * W[2];
        const float gJ02 = gT0[0] * W[6] + gT0[1] * W[7] + gT0[2] * W[8];
        const float gJ11 = gT1[0] * W[3] + gT1[1] * W[4] + gT1[2] * W[5];
        const float gJ12 = gT1[0] * W[6] + gT1[1] * W[7] + gT1[2] * W[8];
        const float tx = p.txf, ty = p.tyf, tz = p.tzf;
        const float iz = 1.0f / tz, iz2 = iz * iz, iz3 = iz2 * iz;
        const float fx = vw.fx, fy = vw.fy;
        float gt[3];
        // J00 = fx/tz; J02 = -fx xi/tz (xi = tx/tz unless clamped); J11, J12 likewise
        gt[0] = p.xclamp ? 0.f : gJ02 * (-fx * iz2);
        gt[1] = p.yclamp ? 0.f : gJ12 * (-fy * iz2);
        gt[2] = -(gJ00 * fx + gJ11 * fy) * iz2 + gJ02 * (p.xclamp ? fx * p.xi * iz2 : 2.f * fx * tx * iz3) +
                gJ12 * (p.yclamp ? fy * p.eta * iz2 : 2.f * fy * ty * iz3);
        // pixel mean u = fx tx / tz + cx, v = fy ty / tz + cy
        gt[0] += gu * fx * iz;
        gt[1] += gv * fy * iz;
        gt[2] -= (gu * fx * tx + gv * fy * ty) * iz2;
        // t = W mu + t_c
        for (int c = 0; c < 3; ++c) gpos[c] += W[c] * gt[0] + W[3 + c] * gt[1] + W[6 + c] * gt[2];
    }

    // The rotation, scales and normalised quaternion are read and formed again here rather than
    // kept in registers through the view loop, which would otherwise spill.
    {
        float pos2[3];
        load_geo(sc, i, pos2, g);
    }
    // S3 = M M', M = Rq diag(s): dL/dM = (G + G') M with G the full symmetric gradient
    // (off-diagonal entries of gS3 hold the sum of both symmetric positions).
    float Gf[9] = {gS3[0], 0.5f * gS3[1], 0.5f * gS3[2], 0.5f * gS3[1], gS3[3], 0.5f * gS3[4],
                   0.5f * gS3[2], 0.5f * gS3[4], gS3[5]};
    float M[9];
    for (int rr = 0; rr < 3; ++rr)
        for (int c = 0; c < 3; ++c) M[3 * rr + c] = g.Rq[3 * rr + c] * g.s[c];
    float gR[9], gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
    if (g.ok) {  // a zero quaternion is culled in every view and gets zero gradients
        for (int rr = 0; rr < 3; ++rr)
            for (int c = 0; c < 3; ++c) {
                const float gM = 2.f * (Gf[3 * rr + 0] * M[c] + Gf[3 * rr + 1] * M[3 + c] + Gf[3 * rr + 2] * M[6 + c]);
                gR[3 * rr + c] = gM * g.s[c];
                gs[c] += gM * g.Rq[3 * rr + c];
            }
        quat_grad(g.qh, gR, gq);
        const float qd = g.qh[0] * gq[0] + g.qh[1] * gq[1] + g.qh[2] * gq[2] + g.qh[3] * gq[3];
        const float iq = 1.0f / g.qnorm;
        for (int c = 0; c < 4; ++c) gq[c] = (gq[c] - g.qh[c] * qd) * iq;
        for (int c = 0; c < 3; ++c) gs[c] *= g.s[c];
    }

    for (int c = 0; c < 3; ++c) G.pos[c * n + i] = gpos[c];
    for (int c = 0; c < 3; ++c) G.logscale[c * n + i] = gs[c];
    for (int c = 0; c < 4; ++c) G.quat[c * n + i] = gq[c];
    G.op_logit[i] = gop;
    if (G.pmask_logit) G.pmask_logit[i] = gpm;
    if constexpr (SHD >= 0) {
#pragma unroll
        for (int m = 0; m < SHM; ++m)
            for (int c = 0; c < 3; ++c) G.sh[((int64_t)m * 3 + c) * n + i] = gsh[m][c];
        return;
    }
    for (int c = 0; c < 3; ++c) G.base[c * n + i] = gbase[c];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        if (RAGGED && l >= lr.cnt) break;
        for (int c = 0; c < 3; ++c) G.axis[lr.at3(l, c)] = gax[l][c];
        G.sharp[lr.at1(l)] = glam[l];
        for (int c = 0; c < 3; ++c) G.amp[lr.at3(l, c)] = gamp[l][c];
        if (G.lmask_logit) G.lmask_logit[lr.at1(l)] = glm[l];
    }
}

// The SG instances run at three waves per SIMD (the compiler keeps them within 168 registers, with
// a few spills, which measured faster than two waves at 209); the SH instances keep their registers.
template <int K, bool RAGGED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_project_bwd(
    SceneDev sc, const ViewInfo* __restrict__ views, int nv, const float* __restrict__ grad2d, GradDev G) {
    project_bwd_one<K, RAGGED, -1>(sc, views, nv, grad2d, G);
}

template <int SHD>
__global__ __launch_bounds__(256) void k_project_bwd_sh(SceneDev sc, const ViewInfo* __restrict__ views, int nv,
                                                        const float* __restrict__ grad2d, GradDev G) {
    project_bwd_one<0, false, SHD>(sc, views, nv, grad2d, G);
}

template <int K, bool RAGGED, int SHD = -1>
hipError_t dispatch_fwd(const SceneDev& sc, const ViewInfo* views, int nv, int tile, const Records& rec,
                        hipStream_t stream) {
    const int64_t blocks = (sc.n + 255) / 256;
    hipLaunchKernelGGL((k_project<K, RAGGED, SHD>), dim3((unsigned)blocks), dim3(256), 0, stream, sc, views, nv, tile, rec);
    return hipGetLastError();
}

template <int K, bool RAGGED, int SHD = -1>
hipError_t dispatch_bwd(const SceneDev& sc, const ViewInfo* views, int nv, const float* grad2d, const GradDev& g,
                        hipStream_t stream) {
    const int64_t blocks = (sc.n + 255) / 256;
    if constexpr (SHD >= 0)
        hipLaunchKernelGGL((k_project_bwd_sh<SHD>), dim3((unsigned)blocks), dim3(256), 0, stream, sc, views, nv,
                           grad2d, g);
    else
        hipLaunchKernelGGL((k_project_bwd<K, RAGGED>), dim3((unsigned)blocks), dim3(256), 0, stream, sc, views, nv,
                           grad2d, g);
    return hipGetLastError();
}

template <bool RAGGED>
hipError_t project_k(const SceneDev& sc, const ViewInfo* views, int nv, int tile, const Records& rec,
                     hipStream_t stream) {
    switch (sc.k) {
        case 0: return dispatch_fwd<0, false>(sc, views, nv, tile, rec, stream);
        case 1: return dispatch_fwd<1, RAGGED>(sc, views, nv, tile, rec, stream);
        case 2: return dispatch_fwd<2, RAGGED>(sc, views, nv, tile, rec, stream);
        case 3: return dispatch_fwd<3, RAGGED>(sc, views, nv, tile, rec, stream);
        case 4: return dispatch_fwd<4, RAGGED>(sc, views, nv, tile, rec, stream);
        case 5: return dispatch_fwd<5, RAGGED>(sc, views, nv, tile, rec, stream);
        case 6: return dispatch_fwd<6, RAGGED>(sc, views, nv, tile, rec, stream);
        case 7: return dispatch_fwd<7, RAGGED>(sc, views, nv, tile, rec, stream);
        case 8: return dispatch_fwd<8, RAGGED>(sc, views, nv, tile, rec, stream);
    }
    return hipErrorInvalidValue;
}

template <bool RAGGED>
hipError_t project_bwd_k(const SceneDev& sc, const ViewInfo* views, int nv, const float* grad2d, const GradDev& g,
                         hipStream_t stream) {
    switch (sc.k) {
        case 0: return dispatch_bwd<0, false>(sc, views, nv, grad2d, g, stream);
        case 1: return dispatch_bwd<1, RAGGED>(sc, views, nv, grad2d, g, stream);
        case 2: return dispatch_bwd<2, RAGGED>(sc, views, nv, grad2d, g, stream);
        case 3: return dispatch_bwd<3, RAGGED>(sc, views, nv, grad2d, g, stream);
        case 4: return dispatch_bwd<4, RAGGED>(sc, views, nv, grad2d, g, stream);
        case 5: return dispatch_bwd<5, RAGGED>(sc, views, nv, grad2d, g, stream);
        case 6: return dispatch_bwd<6, RAGGED>(sc, views, nv, grad2d, g, stream);
        case 7: return dispatch_bwd<7, RAGGED>(sc, views, nv, grad2d, g, stream);
        case 8: return dispatch_bwd<8, RAGGED>(sc, views, nv, grad2d, g, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// A compressed-row scene with k = 0 has no lobes at all and takes the dense k = 0 kernels.
// Spherical-harmonic scenes (sc.sh non-null) take the SH instances, one per degree.
hipError_t launch_project(const SceneDev& sc, const ViewInfo* views, int nv, int tile, const Records& rec,
                          hipStream_t stream) {
    if (sc.n == 0) return hipSuccess;
    if (sc.sh) {
        switch (sc.sh_degree) {
            case 0: return dispatch_fwd<0, false, 0>(sc, views, nv, tile, rec, stream);
            case 1: return dispatch_fwd<0, false, 1>(sc, views, nv, tile, rec, stream);
            case 2: return dispatch_fwd<0, false, 2>(sc, views, nv, tile, rec, stream);
            case 3: return dispatch_fwd<0, false, 3>(sc, views, nv, tile, rec, stream);
        }
        return hipErrorInvalidValue;
    }
    return sc.lobe_off ? project_k<true>(sc, views, nv, tile, rec, stream)
                       : project_k<false>(sc, views, nv, tile, rec, stream);
}

hipError_t launch_project_bwd(const SceneDev& sc, const ViewInfo* views, int nv, const float* grad2d,
                              const GradDev& g, hipStream_t stream) {
    if (sc.n == 0) return hipSuccess;
    if (sc.sh) {
        switch (sc.sh_degree) {
            case 0: return dispatch_bwd<0, false, 0>(sc, views, nv, grad2d, g, stream);
            case 1: return dispatch_bwd<0, false, 1>(sc, views, nv, grad2d, g, stream);
            case 2: return dispatch_bwd<0, false, 2>(sc, views, nv, grad2d, g, stream);
            case 3: return dispatch_bwd<0, false, 3>(sc, views, nv, grad2d, g, stream);
        }
        return hipErrorInvalidValue;
    }
    return sc.lobe_off ? project_bwd_k<true>(sc, views, nv, grad2d, g, stream)
                       : project_bwd_k<false>(sc, views, nv, grad2d, g, stream);
}

}  // namespace megs
