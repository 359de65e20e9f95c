// project.hip -- EWA projection with Spherical-Gaussian colour (forward) and its chain rule
// back to the raw parameters (backward), gfx950.
//
// One thread per Gaussian loops over all views, so the parameter planes are streamed from HBM
// once per launch (coalesced SoA loads, widened from FP16/BF16 in registers) and the records of
// every view are written. View-independent values (activations, 3D covariance, unit lobe axes,
// base colour) are formed once per Gaussian. The camera-space position, the pixel mean and the
// tile count (the row-interval test of the key emission) are computed in FP64, everything else in
// FP32. Each group of parameter loads is issued together (load_n), and the kernels are bound by the
// latency of their dependent arithmetic at the occupancy their registers allow (four waves per SIMD). The forward with SG colour of up to four lobes is
// held to four waves per SIMD (128 registers): left to itself it takes 132 and runs three.
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

// View-independent part: activations and the 3D covariance. The raw quaternion is returned in
// q_raw for load_cov64. The twelve loads are one group (load_n).
__device__ __forceinline__ void load_geo(const SceneDev& sc, int64_t i, float pos[3], Geo& g, float q_raw[4]) {
    const int64_t n = sc.n;
    const void* pl[12];
    int64_t ix[12];
    bool lv[12];
    for (int j = 0; j < 12; ++j) lv[j] = true;
    for (int j = 0; j < 3; ++j) { pl[j] = sc.pos; ix[j] = j * n + i; }
    for (int j = 0; j < 3; ++j) { pl[3 + j] = sc.logscale; ix[3 + j] = j * n + i; }
    for (int j = 0; j < 4; ++j) { pl[6 + j] = sc.quat; ix[6 + j] = j * n + i; }
    pl[10] = sc.op_logit; ix[10] = i;
    pl[11] = sc.pmask_logit; ix[11] = i; lv[11] = sc.pmask_logit != nullptr;
    float f[12];
    load_n(sc.dt_geom, pl, ix, lv, f);
    for (int j = 0; j < 3; ++j) pos[j] = f[j];
    for (int j = 0; j < 3; ++j) g.s[j] = __expf(f[3 + j]);
    float* q = q_raw;
    for (int j = 0; j < 4; ++j) q[j] = f[6 + j];
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
    g.o = sigmoidf(f[10]);
    g.mp = sc.pmask_logit ? sigmoidf(f[11]) : 1.0f;
    g.o_eff = g.o * g.mp;
}

// The 3D covariance's factor M = R(q) diag(s) (Sigma3 = M M'), from which each view projects the
// footprint's shape in FP64: a thin footprint's direction and width must survive the subtraction
// that forms its determinant. Kept across the view loop as the normalised quaternion (FP64) and the
// scales; each view forms the columns of M one at a time (cheaper in registers than holding M).
struct Cov64 {
    double w, x, y, z;
    float s[3];
};

// From the raw quaternion and the scales load_geo formed (the same values it would load again).
__device__ __forceinline__ void load_cov64(const float q_raw[4], const float s[3], Cov64& cv) {
    double q[4], qq = 0.0;
    for (int j = 0; j < 4; ++j) {
        q[j] = (double)q_raw[j];
        qq = fma(q[j], q[j], qq);
    }
    const double inv = 1.0 / sqrt(qq);
    cv.w = q[0] * inv; cv.x = q[1] * inv; cv.y = q[2] * inv; cv.z = q[3] * inv;
    for (int j = 0; j < 3; ++j) cv.s[j] = s[j];
}

// Lobe slots at or past the Gaussian's count get zero mask and amplitude, so they add exactly +0.
// Every lobe's loads are issued before any is converted.
template <int K, bool RAGGED>
__device__ __forceinline__ bool load_lobes(const SceneDev& sc, const LobeRef<RAGGED>& r, Lobes<K>& L) {
    // per lobe: axis (3), sharpness and mask logit in the colour storage type; amplitude (3) in its own.
    // A ragged Gaussian's slots past its count are not read.
    constexpr int KK = K > 0 ? K : 1;
    const void* pc[KK * 5];
    const void* pm[KK * 3];
    int64_t ic[KK * 5], im[KK * 3];
    bool lc[KK * 5], lm[KK * 3];
#pragma unroll
    for (int l = 0; l < KK; ++l) {
        const bool live = l < K && !(RAGGED && l >= r.cnt);
        for (int c = 0; c < 3; ++c) {
            pc[5 * l + c] = sc.axis; ic[5 * l + c] = live ? r.at3(l, c) : 0; lc[5 * l + c] = live;
            pm[3 * l + c] = sc.amp; im[3 * l + c] = live ? r.at3(l, c) : 0; lm[3 * l + c] = live;
        }
        pc[5 * l + 3] = sc.sharp; ic[5 * l + 3] = live ? r.at1(l) : 0; lc[5 * l + 3] = live;
        pc[5 * l + 4] = sc.lmask_logit; ic[5 * l + 4] = live ? r.at1(l) : 0;
        lc[5 * l + 4] = live && sc.lmask_logit != nullptr;
    }
    float fc[KK * 5], fm[KK * 3];
    load_n(sc.dt_color, pc, ic, lc, fc);
    load_n(sc.dt_amp, pm, im, lm, fm);
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
        const float a0 = fc[5 * l], a1 = fc[5 * l + 1], a2 = fc[5 * l + 2];
        float al2 = a0 * a0 + a1 * a1 + a2 * a2;
        const float ia = rsqrtf(al2);
        L.ia[l] = ia;
        L.mu[l][0] = a0 * ia; L.mu[l][1] = a1 * ia; L.mu[l][2] = a2 * ia;
        ok = ok && (al2 > 0.0f) && isfinite(al2);
        L.lam[l] = fc[5 * l + 3];
#pragma unroll
        for (int c = 0; c < 3; ++c) L.amp[l][c] = fm[3 * l + c];
        L.m[l] = sc.lmask_logit ? sigmoidf(fc[5 * l + 4]) : 1.0f;
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
    float T0[3], T1[3];   // rows of J W (FP32 copies for the backward's chain rule)
    double A, B, C, det;  // dilated 2D covariance [[A, B], [B, C]] and its determinant
    float l11, l22;       // the conic's factors as stored (Shape)
    double r;
    int32_t radius;
};

// Camera-space position, pixel mean, the Jacobian's clamp decisions (FP64) and the rows T0, T1 of
// J W: in FP64 for the forward's covariance (T64), and as FP32 copies, which are all the backward's
// chain rule needs. Shared by the forward and the backward, so both take the same decisions.
template <bool T64>
__device__ __forceinline__ void project_cam(const Geo& g, const float pos[3], const ViewInfo& vw, ViewProj& p,
                                            double T0[3], double T1[3]) {
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
    const double rx = p.tx * rz, ry = p.ty * rz, limx = vw.limx, limy = vw.limy;
    p.xclamp = rx < -limx || rx > limx;
    p.yclamp = ry < -limy || ry > limy;
    const double xi = fmin(fmax(rx, -limx), limx), eta = fmin(fmax(ry, -limy), limy);
    p.xi = (float)xi;
    p.eta = (float)eta;
    if constexpr (T64) {
        const double J00 = vw.fx * rz, J02 = -vw.fx * xi * rz;
        const double J11 = vw.fy * rz, J12 = -vw.fy * eta * rz;
        // T = J W: row 0 = J00 W0 + J02 W2, row 1 = J11 W1 + J12 W2
        for (int c = 0; c < 3; ++c) {
            T0[c] = fma(J00, (double)vw.R[c], J02 * vw.R[6 + c]);
            T1[c] = fma(J11, (double)vw.R[3 + c], J12 * vw.R[6 + c]);
            p.T0[c] = (float)T0[c];
            p.T1[c] = (float)T1[c];
        }
    } else {
        const float irz = 1.0f / p.tzf;
        const float J00 = vw.fx * irz, J02 = -vw.fx * p.xi * irz;
        const float J11 = vw.fy * irz, J12 = -vw.fy * p.eta * irz;
        for (int c = 0; c < 3; ++c) {
            p.T0[c] = J00 * vw.R[c] + J02 * vw.R[6 + c];
            p.T1[c] = J11 * vw.R[3 + c] + J12 * vw.R[6 + c];
        }
    }
}

// The forward's projection: project_cam, then the dilated 2D covariance in FP64,
// Sigma2 = (J W M)(J W M)' + h I, formed from the projected scaled axes J W M (so it is positive
// semi-definite before the dilation), det = A C - B^2 >= h^2, its factors (Shape), and the radius.
__device__ __forceinline__ void project_view(const Geo& g, const Cov64& cv, const float pos[3],
                                             const ViewInfo& vw, ViewProj& p) {
    double T0[3], T1[3];
    project_cam<true>(g, pos, vw, p, T0, T1);
    // the projected scaled axes, column c of T M = (T e_c) s_c with e_c column c of R(q), one at a time
    const double w = cv.w, x = cv.x, y = cv.y, z = cv.z;
    double A0 = 0.0, B0 = 0.0, C0 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double e0, e1, e2;
        if (c == 0) {
            e0 = 1.0 - 2.0 * (y * y + z * z); e1 = 2.0 * (x * y + w * z); e2 = 2.0 * (x * z - w * y);
        } else if (c == 1) {
            e0 = 2.0 * (x * y - w * z); e1 = 1.0 - 2.0 * (x * x + z * z); e2 = 2.0 * (y * z + w * x);
        } else {
            e0 = 2.0 * (x * z + w * y); e1 = 2.0 * (y * z - w * x); e2 = 1.0 - 2.0 * (x * x + y * y);
        }
        const double sc = cv.s[c];
        const double p0 = fma(T0[0], e0, fma(T0[1], e1, T0[2] * e2)) * sc;
        const double p1 = fma(T1[0], e0, fma(T1[1], e1, T1[2] * e2)) * sc;
        A0 = fma(p0, p0, A0);
        B0 = fma(p0, p1, B0);
        C0 = fma(p1, p1, C0);
    }
    p.A = A0 + (double)kDilation;
    p.B = B0;
    p.C = C0 + (double)kDilation;
    p.det = fma(p.A, p.C, -p.B * p.B);
    // only the ratio needs FP64 (it carries the footprint's direction); the diagonal factors are
    // stored in FP32 and formed there, from the FP64 covariance rounded once
    p.r = -p.B / p.C;
    const float Cf = (float)p.C, detf = (float)p.det;
    p.l11 = __builtin_amdgcn_sqrtf(Cf / detf);
    p.l22 = __builtin_amdgcn_rsqf(Cf);
    const float rr = ceilf(footprint_rho(p.l11, p.r, p.l22, g.o_eff));
    if (!(isfinite(p.u) && isfinite(p.v) && isfinite(rr)) || fabs(p.u) > kMaxCoord || fabs(p.v) > kMaxCoord ||
        rr > (float)kMaxCoord)
        p.ok = false;
    p.radius = p.ok ? (int32_t)rr : -1;
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
    const void* pl[3] = {sc.base, sc.base, sc.base};
    const int64_t ix[3] = {i, sc.n + i, 2 * sc.n + i};
    const bool lv[3] = {true, true, true};
    float f[3];
    load_n(sc.dt_color, pl, ix, lv, f);
    for (int c = 0; c < 3; ++c) base[c] = f[c];
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
        const void* pl[M];
        int64_t ix[M];
        bool lv[M];
#pragma unroll
        for (int m = 0; m < M; ++m) { pl[m] = sc.sh; ix[m] = ((int64_t)m * 3 + c) * n + i; lv[m] = true; }
        float f[M];  // the channel's coefficients, one group
        load_n(sc.dt_color, pl, ix, lv, f);
        float acc = 0.5f;
#pragma unroll
        for (int m = 0; m < M; ++m) acc = __fmaf_rn(Y[m], f[m], acc);
        clamped[c] = acc < 0.0f;
        rgb[c] = clamped[c] ? 0.0f : acc;
    }
    return isfinite(rgb[0]) && isfinite(rgb[1]) && isfinite(rgb[2]);
}

// Waves per SIMD the forward projection is compiled for: four with SG colour of up to four lobes
// (four lobes fit in 128 registers, and ran 9% faster than at three waves in 132 registers: 0.369 ->
// 0.336 ms on the 8-view 1080p workload), else what its registers give (more lobes and the SH forms
// would spill far more).
template <int K, int SHD>
constexpr int kProjectWaves = (SHD < 0 && K <= 4) ? 4 : 1;

template <int K, bool RAGGED, int SHD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kProjectWaves<K, SHD>))) void k_project(
    SceneDev sc, const ViewInfo* __restrict__ views, int nv, int tile, Records rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.n) return;
    float pos[3];
    Geo g;
    float q_raw[4];
    load_geo(sc, i, pos, g, q_raw);
    Cov64 cv;
    load_cov64(q_raw, g.s, cv);
    Lobes<K> L;
    LobeRef<RAGGED> lr;
    const bool lobes_ok = lobe_ref<RAGGED>(sc, i, K, lr) && load_lobes<K, RAGGED>(sc, lr, L);
    // the forward needs each lobe's mask only as a factor of its amplitude: fold it in once
#pragma unroll
    for (int l = 0; l < K; ++l) {
        for (int c = 0; c < 3; ++c) L.amp[l][c] *= L.m[l];
        L.m[l] = 1.0f;
    }
    float base[3] = {0.f, 0.f, 0.f};
    if constexpr (SHD < 0) load_base(sc, i, base);
    for (int v = 0; v < nv; ++v) {
        const ViewInfo& vw = views[v];
        const int64_t r = (int64_t)v * sc.n + i;
        ViewProj p;
        project_view(g, cv, pos, vw, p);
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
        const float cut = cutoff_of(g.o_eff);
        // the conic the stored factors describe: the key emission and the blend read exactly these
        const Shape shp = shape_of(p.l11, p.r, p.l22);
        if (rec.mean) {  // per-field planes, on request only
            rec.mean[r] = ok ? make_double2(p.u, p.v) : make_double2(0.0, 0.0);
            rec.conic_o[r] = ok ? make_float4((float)shp.a, (float)shp.b, (float)shp.c, g.o_eff)
                                : make_float4(0.f, 0.f, 0.f, 0.f);
            rec.rgbd[r] = ok ? make_float4(rgb[0], rgb[1], rgb[2], p.tzf) : make_float4(0.f, 0.f, 0.f, 0.f);
            rec.radius[r] = ok ? p.radius : -1;
            rec.cutoff[r] = ok ? cut : 0.f;
            rec.chol[r] = ok ? make_double4((double)p.l11, p.r, (double)p.l22, 0.0) : make_double4(0.0, 0.0, 0.0, 0.0);
        }
        // the packed record (what the blend and the projection backward read)
        {
            PackedRec pr;
            pr.mean = ok ? make_double2(p.u, p.v) : make_double2(0.0, 0.0);
            pr.r = ok ? p.r : 0.0;
            pr.l11 = ok ? p.l11 : 0.f;
            pr.l22 = ok ? p.l22 : 0.f;
            pr.o = ok ? g.o_eff : 0.f;
            pr.rgb[0] = ok ? rgb[0] : 0.f;
            pr.rgb[1] = ok ? rgb[1] : 0.f;
            pr.rgb[2] = ok ? rgb[2] : 0.f;
            const float4* src = reinterpret_cast<const float4*>(&pr);
            float4* dst = reinterpret_cast<float4*>(rec.packed + r);
            dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2];
        }
        uint32_t nt = 0;
        if (ok) {
            int x0, x1, y0, y1;
            if (tile_rect(p.u, p.v, p.radius, vw, tile, x0, x1, y0, y1)) {
                EllipseRows er;
                ellipse_rows(p.u, p.v, shp, cut, er);
                for (int ty = y0; ty <= y1; ++ty) {
                    int lo, hi;
                    if (row_span(er, vw.width, vw.height, tile, ty, x0, x1, lo, hi)) nt += (uint32_t)(hi - lo + 1);
                }
            }
        }
        rec.ntiles[r] = nt;
        if (rec.ntiles_plane) rec.ntiles_plane[r] = nt;
        if (sc.status) {  // culled records, one atomic per wave (the lanes here are the wave's Gaussians)
            const uint64_t culled = __ballot(!ok);
            if (culled && __lane_id() == (unsigned)__builtin_ctzll(__ballot(true)))
                atomicAdd(&sc.status[kStatusCulled], (int32_t)__popcll(culled));
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

// The backward runs in two passes over the Gaussians, each looping over the views: the colour pass
// (the colour model's parameters and the colour's share of the position gradient) and then the
// geometry pass (position, scales, rotation, opacity and mask), which adds its share of the position
// gradient to the colour pass's. Each pass keeps only its own state in registers through the view
// loop, and reads its part of the per-record sums the blend leaves ([NR][9]: the six exponent sums,
// then the colour gradient).

// Colour pass. A record whose colour gradient is exactly zero contributes nothing here (every term is
// proportional to it) and is skipped; among them are all records the forward culled.
template <int K, bool RAGGED, int SHD>
__device__ __forceinline__ void project_bwd_colour(const SceneDev& sc, const ViewInfo* __restrict__ views, int nv,
                                                   const float* __restrict__ sums_col, const GradDev& G) {
    constexpr int SHM = SHD >= 0 ? (SHD + 1) * (SHD + 1) : 1;
    float gsh[SHM][3];
#pragma unroll
    for (int m = 0; m < SHM; ++m) gsh[m][0] = gsh[m][1] = gsh[m][2] = 0.f;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.n) return;
    const int64_t n = sc.n;
    float pos[3];
    {
        const void* pl[3] = {sc.pos, sc.pos, sc.pos};
        const int64_t ix[3] = {i, n + i, 2 * n + i};
        const bool lv[3] = {true, true, true};
        load_n(sc.dt_geom, pl, ix, lv, pos);
    }
    Lobes<K> L;
    LobeRef<RAGGED> lr;
    const bool lobes_ok = lobe_ref<RAGGED>(sc, i, K, lr) && load_lobes<K, RAGGED>(sc, lr, L);
    float base[3] = {0.f, 0.f, 0.f};
    if constexpr (SHD < 0) load_base(sc, i, base);
    float gpos[3] = {0.f, 0.f, 0.f}, gbase[3] = {0.f, 0.f, 0.f};
    constexpr int KK = K > 0 ? K : 1;
    float gax[KK][3], glam[KK], gamp[KK][3], glm[KK];
#pragma unroll
    for (int l = 0; l < KK; ++l) {
        gax[l][0] = gax[l][1] = gax[l][2] = 0.f;
        glam[l] = 0.f; glm[l] = 0.f;
        gamp[l][0] = gamp[l][1] = gamp[l][2] = 0.f;
    }
    // each view's three colour sums are loaded one view ahead, so their round trip overlaps the
    // previous view's arithmetic
    float gnext[3] = {0.f, 0.f, 0.f};
    if (nv > 0 && lobes_ok)
        for (int c = 0; c < 3; ++c) gnext[c] = sums_col[9 * i + c];
    for (int v = 0; v < nv && lobes_ok; ++v) {
        const ViewInfo& vw = views[v];
        const float gcol[3] = {gnext[0], gnext[1], gnext[2]};
        if (v + 1 < nv) {
            const int64_t rn = (int64_t)(v + 1) * n + i;
            for (int c = 0; c < 3; ++c) gnext[c] = sums_col[9 * rn + c];
        }
        if (gcol[0] == 0.f && gcol[1] == 0.f && gcol[2] == 0.f) continue;
        float d[3], dlen, rgb[3], e[KK], muh[KK][3], dd2[KK];
        bool clamped[3] = {false, false, false};
        if constexpr (SHD >= 0)
            sh_colour<SHD>(sc, i, pos, vw, d, dlen, rgb, clamped);
        else
            sg_colour<K>(base, pos, vw, L, d, dlen, rgb, e, muh, dd2);
        float gd[3] = {0.f, 0.f, 0.f};
        if constexpr (SHD >= 0) {
            float Y[16], dY[16][3];
            sh_basis<SHD, true>(d, Y, dY);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float gc = clamped[c] ? 0.f : gcol[c];
                const void* pl[SHM];
                int64_t ix[SHM];
                bool lv[SHM];
#pragma unroll
                for (int m = 0; m < SHM; ++m) { pl[m] = sc.sh; ix[m] = ((int64_t)m * 3 + c) * n + i; lv[m] = true; }
                float fsh[SHM];  // the channel's coefficients, one group
                load_n(sc.dt_color, pl, ix, lv, fsh);
#pragma unroll
                for (int m = 0; m < SHM; ++m) {
                    gsh[m][c] = __fmaf_rn(Y[m], gc, gsh[m][c]);
                    const float w = gc * fsh[m];
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
    }
    // the colour's share of the position gradient; the geometry pass adds its own
    for (int c = 0; c < 3; ++c) G.pos[c * n + i] = gpos[c];
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

// Geometry pass: the exponent sums to the pixel mean and the dilated covariance, then through the
// projection to the position, scales, rotation, opacity and mask. Records the forward culled (zero
// factors in the record) are skipped.
__device__ __forceinline__ void project_bwd_geometry(const SceneDev& sc, const ViewInfo* __restrict__ views, int nv,
                                                     const float* __restrict__ sums_exp,
                                                     const PackedRec* __restrict__ rec, const GradDev& G) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.n) return;
    const int64_t n = sc.n;
    float pos[3];
    Geo g;
    float q_raw[4];
    load_geo(sc, i, pos, g, q_raw);
    Cov64 cv;
    load_cov64(q_raw, g.s, cv);
    // H = R' (dL/dSigma3) R, the 3D covariance's gradient in the Gaussian's own axes (xx, xy, xz, yy,
    // yz, zz; full-matrix convention)
    float gpos[3] = {0.f, 0.f, 0.f}, H[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float gop = 0.f, gpm = 0.f;
    // each view's record factors and six exponent sums are loaded one view ahead (all of them, a
    // culled record's included: its sums are zero), so their round trip overlaps the previous view's
    // arithmetic
    float4 fq_next = make_float4(0.f, 0.f, 0.f, 0.f);
    float gr_next[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (nv > 0) {
        fq_next = reinterpret_cast<const float4*>(rec + i)[1];
        for (int c = 0; c < 6; ++c) gr_next[c] = sums_exp[9 * i + c];
    }
    for (int v = 0; v < nv; ++v) {
        const ViewInfo& vw = views[v];
        // the record's conic factors as the forward stored them (zero when the forward culled it)
        const float4 fq = fq_next;
        const float gr[6] = {gr_next[0], gr_next[1], gr_next[2], gr_next[3], gr_next[4], gr_next[5]};
        if (v + 1 < nv) {
            const int64_t rn = (int64_t)(v + 1) * n + i;
            fq_next = reinterpret_cast<const float4*>(rec + rn)[1];
            for (int c = 0; c < 6; ++c) gr_next[c] = sums_exp[9 * rn + c];
        }
        if (!(fq.w > 0.0f)) continue;
        ViewProj p;
        double T0d[3], T1d[3];
        project_cam<true>(g, pos, vw, p, T0d, T1d);
        const float l11 = fq.z, l22 = fq.w;
        const double l21d = (double)l11 * __hiloint2double(__float_as_int(fq.y), __float_as_int(fq.x));
        const float l21 = (float)l21d;
        // The blend leaves, over the record's fragments, e = dL/do_eff of each unclamped fragment and
        // the moments S = sum e w, M = sum e w w' (w1^2, w1 w2, w2^2), then sum e (= dL/do_eff), with
        // w = kQ2 L' d the exponent's factors of the pixel offset d from the mean (conic Q = L L',
        // L = [[l11, 0], [l21, l22]], l21 = l11 r; the exponent is -d' Q d / 2). A fragment's alpha
        // o exp(-d' Q d / 2) has gradient alpha Q d in the mean and (alpha / 2) (Q d)(Q d)' in the
        // dilated covariance Sigma = Q^-1 (from dQ = -Q dSigma Q), and Q d = L w / kQ2, so per record
        //   dL/dmean = (o_eff / kQ2) L S,  dL/dSigma = (o_eff / (2 kQ2^2)) L M L',
        // products of the factors only: no inverse, no determinant, nothing that cancels for a thin
        // footprint.
        const float oe = g.o_eff;
        const float s1 = oe * (1.0f / kQ2), s2 = oe * (0.5f / (kQ2 * kQ2));
        const float gu = s1 * (l11 * gr[0]);
        const float gv = s1 * __fmaf_rn(l21, gr[0], l22 * gr[1]);
        const float t1 = __fmaf_rn(l21, gr[2], l22 * gr[3]);  // sum e w1 (L w)_2
        const float t2 = __fmaf_rn(l21, gr[3], l22 * gr[4]);  // sum e w2 (L w)_2
        const float gA0 = s2 * (l11 * l11 * gr[2]);
        const float gB0 = 2.0f * s2 * (l11 * t1);
        const float gC0 = s2 * __fmaf_rn(l21, t1, l22 * t2);
        const float go = gr[5];
        // opacity and primitive mask
        gop += go * g.mp * g.o * (1.f - g.o);
        gpm += go * g.o * g.mp * (1.f - g.mp);
        // Sigma3's gradient in the Gaussian's axes: with p_c = T R e_c the projected axis c,
        // H_ij += p_i' (dL/dSigma) p_j = s2 q_i' M q_j, q_c = L' p_c. Along a thin footprint the first
        // component of q_c cancels (that is the footprint's direction), so q_c is formed in FP64 from
        // FP64 axes; summing in the axes' frame keeps each axis's own term, which a world-frame sum
        // would bury under the others.
        {
            const double w = cv.w, x = cv.x, y = cv.y, z = cv.z;
            float qv[3][2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double e0, e1, e2;
                if (c == 0) {
                    e0 = 1.0 - 2.0 * (y * y + z * z); e1 = 2.0 * (x * y + w * z); e2 = 2.0 * (x * z - w * y);
                } else if (c == 1) {
                    e0 = 2.0 * (x * y - w * z); e1 = 1.0 - 2.0 * (x * x + z * z); e2 = 2.0 * (y * z + w * x);
                } else {
                    e0 = 2.0 * (x * z + w * y); e1 = 2.0 * (y * z - w * x); e2 = 1.0 - 2.0 * (x * x + y * y);
                }
                const double p0 = fma(T0d[0], e0, fma(T0d[1], e1, T0d[2] * e2));
                const double p1 = fma(T1d[0], e0, fma(T1d[1], e1, T1d[2] * e2));
                qv[c][0] = (float)fma((double)l11, p0, l21d * p1);
                qv[c][1] = (float)((double)l22 * p1);
            }
            float mq[3][2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                mq[c][0] = __fmaf_rn(gr[2], qv[c][0], gr[3] * qv[c][1]);
                mq[c][1] = __fmaf_rn(gr[3], qv[c][0], gr[4] * qv[c][1]);
            }
            H[0] += s2 * __fmaf_rn(qv[0][0], mq[0][0], qv[0][1] * mq[0][1]);
            H[1] += s2 * __fmaf_rn(qv[0][0], mq[1][0], qv[0][1] * mq[1][1]);
            H[2] += s2 * __fmaf_rn(qv[0][0], mq[2][0], qv[0][1] * mq[2][1]);
            H[3] += s2 * __fmaf_rn(qv[1][0], mq[1][0], qv[1][1] * mq[1][1]);
            H[4] += s2 * __fmaf_rn(qv[1][0], mq[2][0], qv[1][1] * mq[2][1]);
            H[5] += s2 * __fmaf_rn(qv[2][0], mq[2][0], qv[2][1] * mq[2][1]);
        }
        const float* T0 = p.T0;
        const float* T1 = p.T1;
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
    // Sigma3 = M M', M = R diag(s): dL/dM = 2 G M with G = dL/dSigma3 = R H R', so
    // dL/dlog s_c = s_c (dL/dM)_{:,c} . R e_c = 2 s_c^2 H_cc and dL/dR = (dL/dM) diag(s) = 2 R H diag(s^2)
    const float Hf[9] = {H[0], H[1], H[2], H[1], H[3], H[4], H[2], H[4], H[5]};
    float gR[9], gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
    if (g.ok) {  // a zero quaternion is culled in every view and gets zero gradients
        for (int c = 0; c < 3; ++c) {
            const float s2c = g.s[c] * g.s[c];
            gs[c] = 2.f * s2c * Hf[4 * c];
            for (int rr = 0; rr < 3; ++rr)
                gR[3 * rr + c] = 2.f * s2c *
                                 (g.Rq[3 * rr] * Hf[c] + g.Rq[3 * rr + 1] * Hf[3 + c] + g.Rq[3 * rr + 2] * Hf[6 + c]);
        }
        quat_grad(g.qh, gR, gq);
        const float qd = g.qh[0] * gq[0] + g.qh[1] * gq[1] + g.qh[2] * gq[2] + g.qh[3] * gq[3];
        const float iq = 1.0f / g.qnorm;
        for (int c = 0; c < 4; ++c) gq[c] = (gq[c] - g.qh[c] * qd) * iq;
    }
    for (int c = 0; c < 3; ++c) G.pos[c * n + i] += gpos[c];  // after the colour pass's share
    for (int c = 0; c < 3; ++c) G.logscale[c * n + i] = gs[c];
    for (int c = 0; c < 4; ++c) G.quat[c * n + i] = gq[c];
    G.op_logit[i] = gop;
    if (G.pmask_logit) G.pmask_logit[i] = gpm;
}

template <int K, bool RAGGED>
__global__ __launch_bounds__(256) void k_project_bwd_col(SceneDev sc, const ViewInfo* __restrict__ views, int nv,
                                                         const float* __restrict__ sums_col, GradDev G) {
    project_bwd_colour<K, RAGGED, -1>(sc, views, nv, sums_col, G);
}

template <int SHD>
__global__ __launch_bounds__(256) void k_project_bwd_sh(SceneDev sc, const ViewInfo* __restrict__ views, int nv,
                                                        const float* __restrict__ sums_col, GradDev G) {
    project_bwd_colour<0, false, SHD>(sc, views, nv, sums_col, G);
}

// held to four waves per SIMD: it fits in 128 registers without spills, where left to itself it takes
// 130 and runs three
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_project_bwd_geo(SceneDev sc, const ViewInfo* __restrict__ views, int nv,
                                                         const float* __restrict__ sums_exp,
                                                         const PackedRec* __restrict__ rec, GradDev G) {
    project_bwd_geometry(sc, views, nv, sums_exp, rec, G);
}

template <int K, bool RAGGED, int SHD = -1>
hipError_t dispatch_fwd(const SceneDev& sc, const ViewInfo* views, int nv, int tile, const Records& rec,
                        hipStream_t stream) {
    const int64_t blocks = (sc.n + 255) / 256;
    hipLaunchKernelGGL((k_project<K, RAGGED, SHD>), dim3((unsigned)blocks), dim3(256), 0, stream, sc, views, nv, tile, rec);
    return hipGetLastError();
}

// colour pass, then geometry pass (which adds to the position gradient the colour pass wrote)
template <int K, bool RAGGED, int SHD = -1>
hipError_t dispatch_bwd(const SceneDev& sc, const ViewInfo* views, int nv, const float* grad2d,
                        const PackedRec* rec, const GradDev& g, hipStream_t stream) {
    const int64_t blocks = (sc.n + 255) / 256;
    const float* sums_exp = grad2d;     // record r's exponent sums at 9 r .. 9 r + 5
    const float* sums_col = grad2d + 6; // its colour gradient at 9 r + 6 .. 9 r + 8
    if constexpr (SHD >= 0)
        hipLaunchKernelGGL((k_project_bwd_sh<SHD>), dim3((unsigned)blocks), dim3(256), 0, stream, sc, views, nv,
                           sums_col, g);
    else
        hipLaunchKernelGGL((k_project_bwd_col<K, RAGGED>), dim3((unsigned)blocks), dim3(256), 0, stream, sc, views, nv,
                           sums_col, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_project_bwd_geo, dim3((unsigned)blocks), dim3(256), 0, stream, sc, views, nv, sums_exp, rec, g);
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
hipError_t project_bwd_k(const SceneDev& sc, const ViewInfo* views, int nv, const float* grad2d,
                         const PackedRec* rec, const GradDev& g, hipStream_t stream) {
    switch (sc.k) {
        case 0: return dispatch_bwd<0, false>(sc, views, nv, grad2d, rec, g, stream);
        case 1: return dispatch_bwd<1, RAGGED>(sc, views, nv, grad2d, rec, g, stream);
        case 2: return dispatch_bwd<2, RAGGED>(sc, views, nv, grad2d, rec, g, stream);
        case 3: return dispatch_bwd<3, RAGGED>(sc, views, nv, grad2d, rec, g, stream);
        case 4: return dispatch_bwd<4, RAGGED>(sc, views, nv, grad2d, rec, g, stream);
        case 5: return dispatch_bwd<5, RAGGED>(sc, views, nv, grad2d, rec, g, stream);
        case 6: return dispatch_bwd<6, RAGGED>(sc, views, nv, grad2d, rec, g, stream);
        case 7: return dispatch_bwd<7, RAGGED>(sc, views, nv, grad2d, rec, g, stream);
        case 8: return dispatch_bwd<8, RAGGED>(sc, views, nv, grad2d, rec, g, stream);
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
                              const PackedRec* rec, const GradDev& g, hipStream_t stream) {
    if (sc.n == 0) return hipSuccess;
    if (sc.sh) {
        switch (sc.sh_degree) {
            case 0: return dispatch_bwd<0, false, 0>(sc, views, nv, grad2d, rec, g, stream);
            case 1: return dispatch_bwd<0, false, 1>(sc, views, nv, grad2d, rec, g, stream);
            case 2: return dispatch_bwd<0, false, 2>(sc, views, nv, grad2d, rec, g, stream);
            case 3: return dispatch_bwd<0, false, 3>(sc, views, nv, grad2d, rec, g, stream);
        }
        return hipErrorInvalidValue;
    }
    return sc.lobe_off ? project_bwd_k<true>(sc, views, nv, grad2d, rec, g, stream)
                       : project_bwd_k<false>(sc, views, nv, grad2d, rec, g, stream);
}

}  // namespace megs
