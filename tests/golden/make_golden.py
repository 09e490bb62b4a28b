"""Write the oracle's reference solutions for the 17-component workload
(unit circle + 16 ellipses, n = 1024, N = 17408) to tests/golden/.

Calls only the CPU oracle (dense FP64 assembly + LU) on the seeded inputs of
the workloads package. Run from the repository root:
    python tests/golden/make_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl            # noqa: E402
from oracle import nystrom as orc  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def main():
    dom, gam = wl.config1()
    g = gam[:, 0]
    t0 = time.time()
    mu, h = orc.fbie(dom.eta, dom.etap, dom.A, g, dom.n)
    t1 = time.time()
    mu_ad = orc.fbiead(dom.eta, dom.etap, dom.etapp, dom.A, dom.Ap, g, dom.n, dom.c)
    t2 = time.time()
    np.savez_compressed(os.path.join(OUT, "cfg1_oracle.npz"), mu=mu, h=h, mu_ad=mu_ad,
                        eta_checksum=np.array([dom.eta.real.sum(), dom.eta.imag.sum()]))
    print(f"fbie {t1 - t0:.1f}s  fbiead {t2 - t1:.1f}s  |mu|={np.abs(mu).max():.3e} "
          f"|h|={np.abs(h).max():.3e} |mu_ad|={np.abs(mu_ad).max():.3e}")


if __name__ == "__main__":
    main()
