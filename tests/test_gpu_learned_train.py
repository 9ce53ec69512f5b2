"""GPU: the learned sensor trained by the library's own kernels on snapshots of
plain-sensor runs of the method (ensemble-type DG problems), and what it gains.

* prediction: on held-out snapshots (other seeds) the trained network's
  mean squared deviation from the plain sensor is below a fifth of the
  untrained network's (same architecture and initial weights);
* accuracy: on an advection problem with an exact solution (periodic shift)
  the learned-sensor run's L1 error is within 10 % of the plain-sensor run's,
  and the purely low-order choice gamma_e = 0 (fixed) is more diffusive
  (larger L1 error) than both;
* determinism: training twice from the same weights and batches gives the
  same weights bit for bit.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw, learned  # noqa: E402


def _snapshots(insts, n, n_snap, every):
    F, G = [], []
    for inst in insts:
        mesh, p, prm, U, dt = synth.instance_case(inst, n=n)
        gm = cvw.Mesh(mesh, p, cvw.DG)
        u = torch.from_numpy(np.asarray(U, np.float32)).cuda()
        sref = learned.sigma_reference(gm, cvw.make_params(prm), u)
        f, g = learned.collect(gm, prm, u, dt, n_snap, every, sref)
        F.append(f)
        G.append(g)
    return torch.cat(F), torch.cat(G)


@pytest.fixture(scope="module")
def trained():
    insts = synth.config5_instances(seed=2005, count=24)
    F, G = _snapshots(insts[:16], 64, 6, 6)
    HF, HG = _snapshots(insts[16:], 64, 4, 8)
    init = learned.init_params(4)
    net = cvw.Mlp(init)
    learned.train(net, F, G, epochs=10, batch=4096, lr=1e-3, seed=4)
    return {"net": net, "init": init, "F": F, "G": G, "HF": HF, "HG": HG}


def test_trained_network_predicts_the_plain_sensor(trained):
    HF, HG = trained["HF"], trained["HG"]
    untrained = cvw.Mlp(trained["init"])
    e_tr = float(((learned.predict(trained["net"], HF) - HG) ** 2).mean())
    e_un = float(((learned.predict(untrained, HF) - HG) ** 2).mean())
    assert (HG < 0.99).float().mean() > 0.05
    assert e_tr < 0.2 * e_un, (e_tr, e_un)


def test_training_is_deterministic(trained):
    a = cvw.Mlp(trained["init"])
    b = cvw.Mlp(trained["init"])
    F, G = trained["F"][:50000], trained["G"][:50000]
    learned.train(a, F, G, epochs=2, batch=1024, seed=11)
    learned.train(b, F, G, epochs=2, batch=1024, seed=11)
    assert np.array_equal(a.get_params(), b.get_params())


def test_learned_sensor_accuracy_on_advection(trained):
    inst = [i for i in synth.config5_instances(seed=3005, count=40) if i.flux == synth.ADVECT_CONST and i.p == 3][0]
    n, steps = 96, 60
    mesh, p, prm, U, dt = synth.instance_case(inst, n=n)
    T = steps * dt
    gq, wq = np.polynomial.legendre.leggauss(p + 1)
    h = 1.0 / n
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    gx, gy = np.meshgrid(gq, gq, indexing="xy")
    X = (ii.ravel() + 0.5)[:, None] * h + 0.5 * h * gx.ravel()[None]
    Y = (jj.ravel() + 0.5)[:, None] * h + 0.5 * h * gy.ravel()[None]
    vx, vy = inst.velocity
    exact = synth.u0_instance(inst, (X - vx * T) % 1.0, (Y - vy * T) % 1.0)
    W = np.outer(wq, wq).ravel() * h * h / 4
    gm = cvw.Mesh(mesh, p, cvw.DG)
    u0 = torch.from_numpy(np.asarray(U, np.float32)).cuda()
    sref = learned.sigma_reference(gm, cvw.make_params(prm), u0)

    def l1(sensor, fixed=1.0, net=None):
        pr = synth.Params(**{**prm.__dict__, "sensor": sensor, "fixed_gamma": fixed})
        cp = cvw.make_params(pr, mlp=net, sigma_ref=sref)
        ws = cvw.alloc_workspace(gm, cp, 1)
        u = u0.clone()
        cvw.step(gm, cp, u, dt, steps, ws)
        assert cvw.poll_status(gm, ws) == 0
        uh = u.cpu().numpy().reshape(-1, (p + 1) ** 2).astype(np.float64)
        return float((np.abs(uh - exact) * W).sum())

    e_plain = l1(0)
    e_learned = l1(cvw.LEARNED, net=trained["net"])
    e_low = l1(2, fixed=0.0)
    assert e_learned <= 1.1 * e_plain, (e_learned, e_plain)
    assert e_low > e_plain and e_low > e_learned, (e_low, e_plain, e_learned)
