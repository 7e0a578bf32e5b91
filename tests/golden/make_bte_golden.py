"""Write the oracle's full-BTE expected values for the diamond 15^3 mesh (C2).

Calls nothing but `oracle/` on the phonons stored in c2_oracle.npz (written
by make_golden.py from the oracle).  Builds every row of the scattering
matrix (Eq. BTE, Eq. gamma1) in worker processes, solves Eq. inverse with a
dense FP64 solve, and keeps:
  gamma0        the diagonal rates [N_q * 3N_b]
  kappa_inv     the conductivity of the inverse [3][3]
  rows_q        a few sampled q-points; rows_val the dense rows of Gamma1 at
                their modes [len(rows_q) * 3N_b][n] (float64, mostly zeros)

    python tests/golden/make_bte_golden.py [workers]   -> tests/golden/c2_bte_oracle.npz
"""
from __future__ import annotations

import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bte  # noqa: E402
from synthetic import configs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROWS_Q = [0, 1, 211, 1687, 3374]
_STATE = {}


def _init():
    g = np.load(os.path.join(HERE, "c2_oracle.npz"))
    cfg = configs.CONFIGS["C2"]
    m = configs.model_for(cfg)
    om, ev, ve = g["omega"], g["evec"], g["vel"]
    st = bte._Setup(m, cfg.mesh, om, ev, cfg.temperature, cfg.broadening)
    _STATE.update(cfg=cfg, model=m, om=om, ev=ev, ve=ve, st=st)


def _rows(qs):
    s = _STATE
    out = []
    for q in qs:
        r0, r1 = bte.scattering_rows(s["model"], s["cfg"].mesh, s["om"], s["ev"], s["ve"],
                                     s["cfg"].temperature, s["cfg"].broadening, q, s["st"])
        nz = np.flatnonzero(np.any(r1 != 0.0, axis=0))
        out.append((q, r0, nz, r1[:, nz]))
    return out


def main(workers=6):
    t0 = time.time()
    _init()
    s = _STATE
    nq, nb3 = s["om"].shape
    n = nq * nb3
    A = np.zeros((n, n))
    g0 = np.zeros(n)
    chunks = [list(range(k, nq, workers * 8)) for k in range(workers * 8)]
    with ProcessPoolExecutor(workers, initializer=_init) as ex:
        for res in ex.map(_rows, chunks):
            for q, r0, nz, vals in res:
                g0[q * nb3:(q + 1) * nb3] = r0
                A[q * nb3:(q + 1) * nb3][:, nz] = vals
    print(f"rows built in {time.time() - t0:.1f} s", flush=True)
    rows = np.concatenate([A[q * nb3:(q + 1) * nb3] for q in ROWS_Q])
    cfg, m = s["cfg"], s["model"]
    act = bte.active_modes(s["om"], g0, cfg.broadening.nu_min_thz)
    lam = bte.solve_inverse(g0, A, s["ve"], act)
    k_inv = bte.kappa_from_lambda(s["om"], s["ve"], lam, cfg.temperature, m.volume, nq, act)
    out = os.path.join(HERE, "c2_bte_oracle.npz")
    np.savez_compressed(out, gamma0=g0, kappa_inv=k_inv, rows_q=np.asarray(ROWS_Q),
                        rows_val=rows)
    print(f"C2 BTE: wrote {out} in {time.time() - t0:.1f} s; kappa_inv diag {np.diag(k_inv)}")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 6)
