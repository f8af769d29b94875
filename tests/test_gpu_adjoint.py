"""GPU adjoint: sky positions and the gradient of the summed squared sky
residual with respect to the initial states, against the CPU oracle's
forward-mode variational equations."""
import math
import sys

import numpy as np
import pytest

from paper_2509_04666_amd import synth

pytestmark = pytest.mark.gpu

MAS = math.radians(1.0 / 3.6e6)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_04666_amd import api
    return torch, api


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _t(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def _setup(torch, api, g, ckpt=5.0, **opts):
    eph = api.DeviceEphemeris.from_synth(g.ephem)
    ctx = api.AdjointContext(eph, g.t0, g.arc, _t(torch, g.t_obs), _t(torch, g.obs_pos), ckpt,
                             api.default_opts(**opts))
    return eph, ctx


def _ang(a, b):
    dra = (a[..., 0] - b[..., 0] + np.pi) % (2 * np.pi) - np.pi
    return np.hypot(dra * np.cos(b[..., 1]), a[..., 1] - b[..., 1])


def test_adjoint_forward_sky_matches_oracle(torch_cuda, orc):
    torch, api = torch_cuda
    g = synth.gradient_case(n_obj=300, k_obs=20, arc=60.0, neo_frac=0.1)
    eph, ctx = _setup(torch, api, g)
    sky = ctx.forward(_t(torch, g.x0)).cpu().numpy()
    st = ctx.status.cpu().numpy()
    radec, loss, grad, ost = orc.sky_grad(g.ephem, g.x0, 0.0, g.t_obs, g.obs_pos, g.radec_obs, want_grad=False)
    np.testing.assert_array_equal(st, ost)
    ok = ost == 0
    assert ok.all()
    diff = _ang(sky, radec)
    diff[~ok] = 0
    err = diff.max()
    _say(f"adjoint forward: max sky difference {err / MAS:.3e} mas")
    worst = np.argsort(diff.max(axis=1))[::-1][:5]
    for j in worst:
        k = int(np.argmax(diff[j]))
        dist = np.linalg.norm(g.x0[j, :3] - g.obs_pos[j, k])
        r = np.linalg.norm(g.x0[j, :3])
        # positions at that observation time, both integrators landing on it
        xs, _, _ = orc.propagate(g.ephem, g.x0[j:j + 1], 0.0, [g.t_obs[j, k]])
        xg, _ = api.propagate(eph, _t(torch, g.x0[j:j + 1]), 0.0, [g.t_obs[j, k]])
        dx = np.abs(xg.cpu().numpy()[0, 0, :3] - xs[0, 0, :3]).max()
        _say(f"  obj {j} obs {k} t={g.t_obs[j, k]:.3f}: {diff[j, k] / MAS:.3e} mas, dist~{dist:.3f} au, "
             f"r~{r:.3f} au, landing-vs-landing |dx| {dx:.2e} au")
    # sky positions agree far inside the 1 mas requirement
    assert err < 1e-3 * MAS
    assert np.median(diff[ok]) < 1e-6 * MAS


def test_adjoint_gradient_matches_oracle_stm(torch_cuda, orc):
    torch, api = torch_cuda
    g = synth.gradient_case(n_obj=200, k_obs=20, arc=60.0, neo_frac=0.1)
    eph, ctx = _setup(torch, api, g)
    x0 = _t(torch, g.x0).requires_grad_(True)
    sky = api.AdjointSky.apply(x0, ctx)
    loss = api.sky_residual_loss(sky, _t(torch, g.radec_obs))
    loss.backward()
    gg = x0.grad.cpu().numpy()
    st = ctx.status.cpu().numpy()
    radec, oloss, og, ost = orc.sky_grad(g.ephem, g.x0, 0.0, g.t_obs, g.obs_pos, g.radec_obs)
    ok = (st == 0) & (ost == 0)
    assert abs(loss.item() - oloss[ok].sum()) <= 1e-9 * oloss[ok].sum() + 1e-30
    rel_x = np.linalg.norm(gg[ok, :3] - og[ok, :3], axis=1) / np.linalg.norm(og[ok, :3], axis=1)
    rel_v = np.linalg.norm(gg[ok, 3:] - og[ok, 3:], axis=1) / np.linalg.norm(og[ok, 3:], axis=1)
    _say(f"adjoint gradient vs oracle STM: max rel (pos) {rel_x.max():.3e}, (vel) {rel_v.max():.3e}, "
         f"median {np.median(rel_x):.3e}")
    assert rel_x.max() < 1e-8 and rel_v.max() < 1e-8


def test_adjoint_gradient_enlarged_j2(torch_cuda, orc):
    # the Jacobian of Eq. A.4 in the discrete adjoint: an oblate Sun with
    # J2 and radius enlarged (a relative force change of about 1e-5 at
    # 2.5 au, 1e-3 further in), about a tilted pole
    import dataclasses
    torch, api = torch_cuda
    g = synth.gradient_case(n_obj=120, k_obs=20, arc=60.0, neo_frac=0.3)
    rng = np.random.default_rng(33)
    pole = rng.normal(size=3)
    pole /= np.linalg.norm(pole)
    g = dataclasses.replace(g, ephem=synth.sun_only_ephemeris(-8.0, g.ephem.coef.shape[1], gr=True,
                                                              j2=(1e-2, 0.05, pole)))
    eph, ctx = _setup(torch, api, g)
    x0 = _t(torch, g.x0).requires_grad_(True)
    sky = api.AdjointSky.apply(x0, ctx)
    loss = api.sky_residual_loss(sky, _t(torch, g.radec_obs))
    loss.backward()
    gg = x0.grad.cpu().numpy()
    st = ctx.status.cpu().numpy()
    radec, oloss, og, ost = orc.sky_grad(g.ephem, g.x0, 0.0, g.t_obs, g.obs_pos, g.radec_obs)
    np.testing.assert_array_equal(st, ost)
    ok = st == 0
    rel = np.linalg.norm(gg[ok] - og[ok], axis=1) / np.linalg.norm(og[ok], axis=1)
    _say(f"enlarged J2 adjoint gradient vs oracle STM: max rel {rel.max():.3e}")
    assert ok.sum() > 100 and rel.max() < 1e-8


def test_adjoint_gradient_sixteen_perturbers(torch_cuda, orc):
    # the most perturbers the ABI takes (run-time body count path of the
    # forward, recompute and sweep kernels)
    import dataclasses
    torch, api = torch_cuda
    g = synth.gradient_case(n_obj=120, k_obs=20, arc=60.0, neo_frac=0.1)
    model = synth.PlanetModel.make(synth.PLANET_NAMES + synth.ASTEROID_NAMES, moon=False)
    g = dataclasses.replace(g, ephem=synth.make_ephemeris(model, -8.0, g.ephem.coef.shape[1]))
    assert g.ephem.coef.shape[0] == 16
    eph, ctx = _setup(torch, api, g)
    x0 = _t(torch, g.x0).requires_grad_(True)
    sky = api.AdjointSky.apply(x0, ctx)
    loss = api.sky_residual_loss(sky, _t(torch, g.radec_obs))
    loss.backward()
    gg = x0.grad.cpu().numpy()
    st = ctx.status.cpu().numpy()
    radec, oloss, og, ost = orc.sky_grad(g.ephem, g.x0, 0.0, g.t_obs, g.obs_pos, g.radec_obs)
    ok = (st == 0) & (ost == 0)
    assert ok.all()
    dsky = _ang(sky.detach().cpu().numpy(), radec)[ok].max()
    rel = np.linalg.norm(gg[ok] - og[ok], axis=1) / np.linalg.norm(og[ok], axis=1)
    _say(f"16 perturbers: max sky difference {dsky / MAS:.3e} mas, max rel gradient difference {rel.max():.3e}")
    assert dsky < 1e-3 * MAS
    assert rel.max() < 1e-8


def test_adjoint_checkpoint_interval_invariance(torch_cuda):
    torch, api = torch_cuda
    g = synth.gradient_case(n_obj=150, k_obs=12, arc=60.0, neo_frac=0.1)
    x0 = _t(torch, g.x0)
    grads = []
    for ckpt in (5.0, 13.0, 60.0):
        eph, ctx = _setup(torch, api, g, ckpt, adj_seg_steps=256)
        sky = ctx.forward(x0)
        dsky = torch.ones_like(sky) * 1e-3
        grads.append(ctx.backward(x0, dsky).cpu().numpy())
        assert int((ctx.status != 0).sum()) == 0
    for k in (1, 2):
        rel = np.linalg.norm(grads[k] - grads[0], axis=1) / np.linalg.norm(grads[0], axis=1)
        _say(f"checkpoint interval invariance: max rel {rel.max():.3e}")
        assert rel.max() < 1e-9


def test_adjoint_failed_objects_get_zero_gradient(torch_cuda):
    torch, api = torch_cuda
    g = synth.gradient_case(n_obj=70, k_obs=5, arc=20.0)
    x0 = g.x0.copy()
    x0[3] = np.nan
    eph, ctx = _setup(torch, api, g)
    xt = _t(torch, x0)
    sky = ctx.forward(xt)
    assert ctx.status[3].item() != 0
    grad = ctx.backward(xt, torch.ones_like(sky))
    assert torch.all(grad[3] == 0)
    assert torch.all(torch.isfinite(grad[torch.arange(70, device="cuda") != 3]))
