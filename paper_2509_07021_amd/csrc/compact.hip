// compact.hip -- the post-processing of Sec. 3.3 (post-processing procedure), gfx950: Gaussians whose
// opacity is below a threshold are dropped, lobes whose sharpness is below a threshold are dropped
// and their sphere mean is folded into the base colour (the compensation equation; Appendix,
// derivation of the colour compensation: delta c0 = m a (1 - e^{-2s}) / (2s), the average of the
// lobe over all directions), and what remains is written as a compressed-row scene whose Gaussians
// own 0..k lobes each.
//
// Two streaming passes over the parameter planes (HBM-bound, one thread per Gaussian, coalesced SoA
// reads): a mark pass that takes the keep decisions and counts the kept lobes, two exclusive scans
// that turn them into output positions, and a write pass that gathers each kept Gaussian into its
// slot. Kept Gaussians and kept lobes are a subsequence of the input, so the writes of a wave land
// in a narrow window and coalesce too. Decisions and the compensation sum are taken in FP64 from the
// stored values; each output value is rounded once to FP32 and then to its storage dtype. Planes
// that need no arithmetic (position, scale, rotation, axis, sharpness) are copied bit for bit.
#include "megs_internal.hpp"

namespace megs {
namespace {

__device__ __forceinline__ double sigmoid_d(double x) { return 1.0 / (1.0 + exp(-x)); }

// (1 - e^{-2s}) / (2s): the mean of e^{s (mu . d - 1)} over the unit sphere; 1 at s = 0.
__device__ __forceinline__ double sphere_mean(double s) { return s == 0.0 ? 1.0 : -expm1(-2.0 * s) / (2.0 * s); }

// logit(sigmoid(a) sigmoid(b)) = -log(e^-a + e^-b + e^-(a+b)), evaluated around the largest term.
__device__ __forceinline__ double folded_logit(double a, double b) {
    const double t1 = -a, t2 = -b, t3 = -a - b;
    const double m = fmax(t1, fmax(t2, t3));
    return -(m + log(exp(t1 - m) + exp(t2 - m) + exp(t3 - m)));
}

template <bool RAGGED>
__global__ __launch_bounds__(256) void k_compact_mark(CompactArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.in.n) return;
    const SceneDev& sc = a.in;
    LobeRef<RAGGED> lr;
    const bool ok = lobe_ref<RAGGED>(sc, i, sc.k, lr);
    const double o = sigmoid_d(load_elem(sc.op_logit, sc.dt_geom, i)) *
                     (sc.pmask_logit ? sigmoid_d(load_elem(sc.pmask_logit, sc.dt_geom, i)) : 1.0);
    const bool keep = ok && o >= a.opacity_min;
    uint32_t cnt = 0;
    if (keep)
        for (int l = 0; l < lr.cnt; ++l) cnt += (double)load_elem(sc.sharp, sc.dt_color, lr.at1(l)) >= a.sharp_min;
    a.keep[i] = keep;
    a.count[i] = cnt;
}

template <bool RAGGED>
__global__ __launch_bounds__(256) void k_compact_write(CompactArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.in.n || !a.keep[i]) return;
    const SceneDev& sc = a.in;
    const int64_t n = sc.n, no = a.n_out, lo = a.l_out;
    const int64_t j = a.new_idx[i];
    LobeRef<RAGGED> lr;
    lobe_ref<RAGGED>(sc, i, sc.k, lr);  // validated by the mark pass (the Gaussian is kept)

    for (int c = 0; c < 3; ++c) copy_elem(a.pos, c * no + j, sc.pos, c * n + i, sc.dt_geom);
    for (int c = 0; c < 3; ++c) copy_elem(a.logscale, c * no + j, sc.logscale, c * n + i, sc.dt_geom);
    for (int c = 0; c < 4; ++c) copy_elem(a.quat, c * no + j, sc.quat, c * n + i, sc.dt_geom);
    if (sc.pmask_logit)
        store_elem(a.op_logit, sc.dt_geom, j,
                   (float)folded_logit(load_elem(sc.op_logit, sc.dt_geom, i), load_elem(sc.pmask_logit, sc.dt_geom, i)));
    else
        copy_elem(a.op_logit, j, sc.op_logit, i, sc.dt_geom);

    double base[3];
    for (int c = 0; c < 3; ++c) base[c] = load_elem(sc.base, sc.dt_color, c * n + i);
    const int64_t d0 = a.lobe_pos[i];
    int64_t d = d0;
    for (int l = 0; l < lr.cnt; ++l) {
        const double s = load_elem(sc.sharp, sc.dt_color, lr.at1(l));
        const double m = sc.lmask_logit ? sigmoid_d(load_elem(sc.lmask_logit, sc.dt_color, lr.at1(l))) : 1.0;
        if (s >= a.sharp_min) {
            for (int c = 0; c < 3; ++c) copy_elem(a.axis, c * lo + d, sc.axis, lr.at3(l, c), sc.dt_color);
            copy_elem(a.sharp, d, sc.sharp, lr.at1(l), sc.dt_color);
            for (int c = 0; c < 3; ++c) {
                if (sc.lmask_logit)
                    store_elem(a.amp, sc.dt_amp, c * lo + d, (float)(m * load_elem(sc.amp, sc.dt_amp, lr.at3(l, c))));
                else
                    copy_elem(a.amp, c * lo + d, sc.amp, lr.at3(l, c), sc.dt_amp);
            }
            a.lobe_src[d] = (int32_t)(RAGGED ? lr.off + l : (int64_t)l * n + i);
            ++d;
        } else {
            const double g = m * sphere_mean(s);
            for (int c = 0; c < 3; ++c) base[c] += g * load_elem(sc.amp, sc.dt_amp, lr.at3(l, c));
        }
    }
    for (int c = 0; c < 3; ++c) store_elem(a.base, sc.dt_color, c * no + j, (float)base[c]);
    a.kept[j] = (int32_t)i;
    a.lobe_off[j] = (int32_t)d0;
}

inline unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_compact_mark(const CompactArgs& a, hipStream_t stream) {
    if (a.in.n == 0) return hipSuccess;
    if (a.in.lobe_off)
        hipLaunchKernelGGL(k_compact_mark<true>, dim3(blocks_of(a.in.n)), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(k_compact_mark<false>, dim3(blocks_of(a.in.n)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_compact_write(const CompactArgs& a, hipStream_t stream) {
    if (a.in.n == 0 || a.n_out == 0) return hipSuccess;
    if (a.in.lobe_off)
        hipLaunchKernelGGL(k_compact_write<true>, dim3(blocks_of(a.in.n)), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(k_compact_write<false>, dim3(blocks_of(a.in.n)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace megs
