"""The paper's flow past a circular cylinder run to a developed state on the
GPU (FP64, cell order kept between sorts), against the coefficients the paper
prints (tests/golden/cylinder_coefficients.json, Sec. 4.6):

* Re = 20 at the coarsest spacing of Table table:hybridconv (dx = 0.10,
  97k particles, 100 s = 36.7k steps), hybrid and modified do-nothing
  outlets: the steady drag coefficient within 1% of the printed value (the
  paper's own values vary by 0.2% over its three spacings; its inlet and
  the placement of its body particles are not specified to the detail that
  would make closer agreement meaningful);
* Re = 200 at the paper's spacing (dx = 0.0667, 212k particles, 150 s =
  55k steps), hybrid outlet: the mean drag over 100 to 150 s inside the
  printed band 1.524 +- 0.05 and the Strouhal number of the lift within 0.015
  of the printed 0.210. The lift amplitude is reported (measured about 0.9
  against the printed 0.722; the paper's five-point filter and averaging are
  not specified).

Coefficients are F / (0.5 rho u^2 D) per unit depth, F the force on the body.
"""
import json
import os

import numpy as np
import pytest

from paper_1907_04034_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "cylinder_coefficients.json")))


def _run(dx, Re, outlet, T):
    from paper_1907_04034_amd import binding as B
    prm, s = I.cylinder_tunnel(dx=dx, Re=Re, outlet=I.OUTLETS[outlet])
    prm["flags"] |= I.FLAG_REUSE_BINS
    sim = B.Simulation(prm, s)
    nwin = int(round(10.0 / prm["dt"]))
    out = []
    for w in range(int(round(T / 10.0))):
        dh = torch.zeros((nwin, 3), dtype=torch.float64, device="cuda")
        sim.step(nwin, drag_hist=dh)
        out.append(dh.cpu().numpy())
        assert sim.poll_error() == 0
        print(f"  t = {(w + 1) * 10} s", flush=True)
    h = np.concatenate(out)
    D = 2.0
    coef = h[:, :2] / (0.5 * prm["rho0"] * prm["U"] ** 2 * D)
    t = (np.arange(len(h)) + 1) * prm["dt"]
    return t, coef, prm["dt"]


@pytest.mark.parametrize("outlet", ["hybrid", "mod-do-nothing"])
def test_cylinder_re20_drag_matches_paper(outlet):
    print(f"cylinder Re 20 dx 0.10 {outlet}", flush=True)
    t, coef, _ = _run(0.10, 20.0, outlet, 100.0)
    cd = coef[t > 60.0, 0].mean()
    ref = GOLDEN["re20_cd"][outlet]["0.10"]
    print(f"  c_d = {cd:.4f} (paper {ref})", flush=True)
    assert abs(cd - ref) <= 0.01 * ref


def test_cylinder_re200_drag_and_strouhal_match_paper():
    print("cylinder Re 200 dx 0.0667 hybrid", flush=True)
    t, coef, dt = _run(0.0667, 200.0, "hybrid", 150.0)
    ref = GOLDEN["re200"]["hybrid"]
    m = t > 100.0
    cd = coef[m, 0].mean()
    cl = coef[m, 1] - coef[m, 1].mean()
    f = np.fft.rfftfreq(len(cl), dt)
    spec = np.abs(np.fft.rfft(cl))
    st = f[1 + np.argmax(spec[1:])] * 2.0 / 1.0
    amp = np.abs(np.convolve(coef[m, 1], np.ones(5) / 5, "valid")).max()
    print(f"  c_d = {cd:.4f} (paper {ref['cd']} +- {ref['cd_band']}), St = {st:.4f} "
          f"(paper {ref['st']}), c_l amplitude {amp:.3f} (paper {ref['cl_amplitude']})",
          flush=True)
    assert abs(cd - ref["cd"]) <= ref["cd_band"]
    assert abs(st - ref["st"]) <= 0.015
    assert 0.5 * ref["cl_amplitude"] < amp < 1.5 * ref["cl_amplitude"]
