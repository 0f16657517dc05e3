"""The constants the paper states (tests/golden/paper_parameters.txt, each
with its citation) are the defaults of the library and of the oracle, and
the oracle's blend window has the stated size."""
import os

import numpy as np

import oracle
from paper_2106_08034_amd import wrls

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    vals = {}
    for line in open(os.path.join(HERE, "golden", "paper_parameters.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            name, value = line.split()[:2]
            vals[name] = float(value)
    return vals


def test_library_defaults_are_the_papers():
    g = _golden()
    p = wrls.wrls_params_default(64, 48, int(g["paper_d"]))
    assert abs(p.alpha - g["alpha"]) < 1e-7 and abs(p.h - g["h"]) < 1e-7
    p.weight_mode = wrls.WRLS_W_PAPER
    assert wrls.wrls_params_validate(p) == wrls.WRLS_OK
    p.d = int(g["paper_d"]) + 1
    assert wrls.wrls_params_validate(p) == wrls.WRLS_EINVAL
    q = wrls.wrls_params_default(64, 48, 8)
    q.lambda_ = g["lambda_example"]
    assert wrls.wrls_params_validate(q) == wrls.WRLS_OK


def test_oracle_defaults_and_blend_window_are_the_papers():
    g = _golden()
    import inspect
    sig = inspect.signature(oracle.Oracle.__init__)
    assert sig.parameters["alpha"].default == g["alpha"]
    assert sig.parameters["h_bw"].default == g["h"]
    # a single non-zero model at the centre reaches exactly the pixels of
    # the blend window around it (sigma_s = inf, no range term)
    n = int(g["blend_window"])
    W = H = 2 * n + 1
    beta = np.zeros((3, 1, H, W))
    beta[:, 0, n, n] = 1.0
    o = oracle.Oracle(W, H, 1)
    o.set_state(np.ones((1, 1, H, W)), beta, frames=1)
    out = o.blend(None, np.inf, np.inf)
    reach = np.argwhere(out[0] > 0)
    assert reach[:, 0].min() == n - n // 2 and reach[:, 0].max() == n + n // 2
    assert reach[:, 1].min() == n - n // 2 and reach[:, 1].max() == n + n // 2
