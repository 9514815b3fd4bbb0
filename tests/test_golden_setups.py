"""The paper's own test setups (tests/golden/paper_setups.json, each with its
citation) run through the oracle: the qualitative results the paper states
for them -- VGF far more accurate than HE at the same N, HE second order."""
import json
import os

import numpy as np

from paper_2103_08531_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_paper_setups_vgf_beats_he(orc):
    setups = json.load(open(os.path.join(HERE, "golden", "paper_setups.json")))["setups"]
    for s in setups:
        if "sigma" not in s:
            continue
        dim, sig = s["dim"], s["sigma"]
        lo, hi = s["domain"]
        for N in ((20, 40) if dim == 2 else (20, 30)):
            n, h, x0 = W.cube_grid(dim, N, lo, hi)
            c = np.zeros((1, dim))
            sg = np.full((1, dim), sig)
            rho = W.gaussian_density(n, x0, h, c, sg, np.ones(1))
            pa, _ = orc.gauss_mixture_grid(n, x0, h, c, sg, np.ones(1), want_E=False)
            pv, _ = orc.solve_fft2n(n, h, orc.kernel("vgf", n, h), rho, want_E=False)
            ph, _ = orc.solve_fft2n(n, h, orc.kernel("he", n, h), rho, want_E=False)
            ev = np.max(np.abs((pv - pa) / pa))  # the paper's metric, Eq. 12
            eh = np.max(np.abs((ph - pa) / pa))
            assert ev < eh / 10, (s["cite"], N, ev, eh)
