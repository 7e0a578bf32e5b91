"""Write oracle-only expected values for the full-size parity tests.

Calls nothing but `oracle/` and the seeded inputs of `synthetic/`.

Crystal configs (C2, C3): the oracle's own phonons (omega, eta, v), its FP64
linewidths for every mode and the RTA conductivity, so the GPU path can be fed
exactly the same eigenvectors.

Gamma-point config (C4): the oracle's real eigenproblem (LAPACK) gives omega
and E; the file keeps omega and the FP64 linewidths of every mode (E, 19 MB,
is recomputed by the test with the same oracle call and checked against the
stored omega; degenerate clusters are compared as sums, which do not depend
on the basis chosen inside a cluster).

    python tests/golden/make_golden.py C2      -> tests/golden/c2_oracle.npz
    python tests/golden/make_golden.py C3      -> tests/golden/c3_oracle.npz
    python tests/golden/make_golden.py C4      -> tests/golden/c4_oracle.npz
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
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    c = configs.CONFIGS[cfg_name]
    m = configs.model_for(c)
    if c.mesh == (1, 1, 1):
        om, E = phonons.phonons_gamma_real(m)
        _STATE.update(cfg=c, model=m, om=om, E=E)
    else:
        om, ev, ve = phonons.phonons(m, c.mesh)
        _STATE.update(cfg=c, model=m, om=om, ev=ev, ve=ve)


def _rows(qs):
    s = _STATE
    G = linewidths.crystal_linewidths(s["model"], s["cfg"].mesh, s["om"], s["ev"], s["ve"],
                                      s["cfg"].temperature, s["cfg"].broadening, q_list=qs)
    return qs, G[qs]


def _modes(ms):
    s = _STATE
    G = linewidths.gamma_point_linewidths(s["model"], s["om"], s["E"], s["cfg"].temperature,
                                          s["cfg"].broadening, modes=ms)
    return ms, G[ms]


def main(cfg_name, workers=8):
    t0 = time.time()
    _init(cfg_name)
    c, m = _STATE["cfg"], _STATE["model"]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{cfg_name.lower()}_oracle.npz")
    if c.mesh == (1, 1, 1):
        om = _STATE["om"]
        n = len(om)
        chunks = [list(range(k, n, workers * 4)) for k in range(workers * 4)]
        G = np.full(n, np.nan)
        with ProcessPoolExecutor(workers, initializer=_init, initargs=(cfg_name,)) as ex:
            for ms, rows in ex.map(_modes, chunks):
                G[ms] = rows
        np.savez_compressed(out, omega=om, gamma=G)
        print(f"{cfg_name}: wrote {out} in {time.time() - t0:.1f} s; max Gamma {G.max():.6e}")
        return
    om, ev, ve = _STATE["om"], _STATE["ev"], _STATE["ve"]
    nq = om.shape[0]
    chunks = [list(range(k, nq, workers * 4)) for k in range(workers * 4)]
    G = np.full(om.shape, np.nan)
    with ProcessPoolExecutor(workers, initializer=_init, initargs=(cfg_name,)) as ex:
        for qs, rows in ex.map(_rows, chunks):
            G[qs] = rows
    k = kappa.kappa_rta(om, ve, G, c.temperature, m.volume, nq, c.broadening.nu_min_thz)
    np.savez_compressed(out, omega=om, evec=ev, vel=ve, gamma=G, kappa=k)
    print(f"{cfg_name}: wrote {out} in {time.time() - t0:.1f} s; kappa diag {np.diag(k)}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "C2",
         int(sys.argv[2]) if len(sys.argv) > 2 else 8)
