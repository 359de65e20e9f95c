"""GPU parity of the training-step pieces against the FP64 oracle: the 3DGS photometric loss and
its gradient (ragged and full-size images), the Adam step in every storage dtype, and a short
self-fit run that closes the loop (render, loss, backward, Adam)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S
from paper_2509_07021_amd import train as T

from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


class _Size:
    def __init__(self, w, h):
        self.width, self.height = w, h


def _loss_case(sizes, seed, lam=0.2):
    rng = np.random.default_rng(seed)
    xs = [rng.uniform(-0.1, 1.1, size=(3, h, w)).astype(np.float32) for w, h in sizes]
    ys = [np.clip(x + rng.normal(0, 0.15, size=x.shape), 0, 1).astype(np.float32) for x in xs]
    ys[0][:, :4, :4] = xs[0][:, :4, :4]                    # some pixels with x = y exactly
    cams = [_Size(w, h) for w, h in sizes]
    flat = lambda a: torch.from_numpy(np.concatenate([v.reshape(-1) for v in a])).cuda()
    log(f"loss case sizes={sizes}")
    loss, dl = T.photometric_loss(flat(xs), flat(ys), cams, lam)
    torch.cuda.synchronize()
    ref, grads = O.photometric_loss([x.astype(np.float64) for x in xs], [y.astype(np.float64) for y in ys], lam)
    np.testing.assert_allclose(float(loss), ref, rtol=1e-12)
    got = dl.cpu().numpy().astype(np.float64)
    want = np.concatenate([g.reshape(-1) for g in grads])
    bound = 2.0 ** -23 * np.abs(want) + 1e-12 * np.abs(want).max()
    assert np.all(np.abs(got - want) <= bound), float((np.abs(got - want) / bound).max())


def test_loss_ragged_views():
    _loss_case([(37, 29), (64, 48), (5, 3)], 130)


def test_loss_pure_terms():
    _loss_case([(40, 33)], 131, lam=0.0)
    _loss_case([(40, 33)], 132, lam=1.0)


def test_loss_full_hd():
    _loss_case([(1920, 1080)], 133)


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_adam_matches_oracle(dt):
    rng = np.random.default_rng(134)
    n = 100_003
    p32 = rng.normal(size=n).astype(np.float32)
    stored = S.to_storage(p32, dt)
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dt]
    if dt == "bf16":
        p = torch.from_numpy(stored.view(np.int16)).view(torch.bfloat16).cuda()
    else:
        p = torch.from_numpy(stored).cuda()
    m = torch.zeros(n, device="cuda")
    v = torch.zeros(n, device="cuda")
    ref_p = S.widen(stored, dt).astype(np.float64)
    m_host = v_host = None
    lib = T.L.load()
    code = {"f32": T.L.MEGS_F32, "f16": T.L.MEGS_F16, "bf16": T.L.MEGS_BF16}[dt]
    ulp = {"f32": 2.0 ** -23, "f16": 2.0 ** -10, "bf16": 2.0 ** -7}[dt]
    for step in (1, 2, 3):
        g32 = rng.normal(size=n).astype(np.float32)
        g = torch.from_numpy(g32).cuda()
        T.L.check(lib.megs_adam_step(n, p.data_ptr(), code, g.data_ptr(), m.data_ptr(), v.data_ptr(), 1e-2, 0.9,
                                     0.999, 1e-15, step, torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        # the kernel receives the hyperparameters as FP32 values; the oracle takes the same values
        f = lambda x: float(np.float32(x))
        prev_m = m_host if step > 1 else np.zeros(n)
        new_p, ref_m, ref_v = O.adam_step(ref_p, g32, prev_m, v_host if step > 1 else np.zeros(n), f(1e-2), f(0.9),
                                          f(0.999), f(1e-15), step)
        m_host = m.cpu().numpy().astype(np.float64)
        v_host = v.cpu().numpy().astype(np.float64)
        # FP32 rounding of a sum errs relative to its terms, which cancel where m crosses zero
        m_terms = f(0.9) * np.abs(prev_m) + (1 - f(0.9)) * np.abs(g32)
        assert np.all(np.abs(m_host - ref_m) <= 3e-7 * m_terms + 1e-30)
        np.testing.assert_allclose(v_host, ref_v, rtol=1e-6, atol=1e-30)
        got = p.float().cpu().numpy().astype(np.float64)
        # one storage ulp for the final rounding plus FP32 rounding of the update
        assert np.all(np.abs(got - new_p) <= ulp * np.abs(new_p) + 1e-5 * 1e-2 + 1e-30)
        ref_p = got            # continue both sides from the stored values
        assert p.dtype == tdt


def test_self_fit_loss_decreases():
    """Targets rendered from a scene; start from perturbed colours and opacities; 150 steps of
    render, loss, backward and Adam must cut the loss by more than half."""
    rng = np.random.default_rng(135)
    truth = S.random_scene(rng, 3000, 3, masks=False, spread=1.0, logscale_mu=-3.0)
    cams = [S.look_at((0.3, -3.5, 0.6), 128, 96), S.look_at((2.5, 2.0, 1.2), 96, 128)]
    ds_t = R.DeviceScene.from_scene(truth)
    targets = R.forward(ds_t, cams, R.Config()).images.clone()
    start = S.Scene(**{f: getattr(truth, f) for f in ("n", "k", "pos", "logscale", "quat", "op_logit",
                                                       "pmask_logit", "base", "axis", "sharp", "amp",
                                                       "lmask_logit")})
    start.base = np.clip(truth.base + rng.normal(0, 0.3, size=truth.base.shape), 0, 1).astype(np.float32)
    start.op_logit = (truth.op_logit + rng.normal(0, 1.0, size=truth.n)).astype(np.float32)
    ds = R.DeviceScene.from_scene(start)
    opt = T.Adam(ds, lr={"base": 2e-2, "op_logit": 5e-2, "pos": 0.0, "logscale": 0.0, "quat": 0.0, "axis": 0.0,
                         "sharp": 0.0, "amp": 1e-2})
    losses = []
    for it in range(150):
        losses.append(float(T.train_step(ds, cams, targets, opt)))
    log(f"self-fit loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
