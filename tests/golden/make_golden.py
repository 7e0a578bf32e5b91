"""Write oracle-only expected values for the full-size parity tests.

Calls nothing but `oracle/` and the seeded inputs of `synthetic/`: the oracle's
own phonons (omega, eta, v) and its FP64 linewidths for every mode, so the GPU
path can be fed exactly the same eigenvectors.

    python tests/golden/make_golden.py C2      -> tests/golden/c2_oracle.npz
"""
from __future__ import annotations

import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import kappa, linewidths, phonons  # noqa: E402
from synthetic import configs  # noqa: E402

_STATE = {}


def _init(cfg_name):
    c = configs.CONFIGS[cfg_name]
    m = configs.model_for(c)
    om, ev, ve = phonons.phonons(m, c.mesh)
    _STATE.update(cfg=c, model=m, om=om, ev=ev, ve=ve)


def _rows(qs):
    s = _STATE
    G = linewidths.crystal_linewidths(s["model"], s["cfg"].mesh, s["om"], s["ev"], s["ve"],
                                      s["cfg"].temperature, s["cfg"].broadening, q_list=qs)
    return qs, G[qs]


def main(cfg_name, workers=8):
    t0 = time.time()
    _init(cfg_name)
    c, m = _STATE["cfg"], _STATE["model"]
    om, ev, ve = _STATE["om"], _STATE["ev"], _STATE["ve"]
    nq = om.shape[0]
    chunks = [list(range(k, nq, workers * 4)) for k in range(workers * 4)]
    G = np.full(om.shape, np.nan)
    with ProcessPoolExecutor(workers, initializer=_init, initargs=(cfg_name,)) as ex:
        for qs, rows in ex.map(_rows, chunks):
            G[qs] = rows
    k = kappa.kappa_rta(om, ve, G, c.temperature, m.volume, nq, c.broadening.nu_min_thz)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{cfg_name.lower()}_oracle.npz")
    np.savez_compressed(out, omega=om, evec=ev, vel=ve, gamma=G, kappa=k)
    print(f"{cfg_name}: wrote {out} in {time.time() - t0:.1f} s; kappa diag {np.diag(k)}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "C2")
