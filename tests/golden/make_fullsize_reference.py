"""Write the FP64 oracle reference of the benchmark workload's first load
step (L = 4096, f = 0.3, seed 0, simple shear E = (0, 0, 0.1), reference
medium C0_SOFT x matrix), iteration-locked over ITERS iterations, sampled at
NSAMP pixels drawn with a fixed seed.  Calls only the oracle and the shared
input generator; a converged or iteration-locked FP64 CPU solve at this size
takes minutes, too long for a test, so the GPU test reads this file.

    python tests/golden/make_fullsize_reference.py   (about 10-20 minutes, ~25 GB)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import alm  # noqa: E402
from paper_0802_2488_amd import synth  # noqa: E402

L, F, SEED, ITERS, NSAMP = 4096, 0.3, 0, 20, 8192
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_L4096_shear_step1.npz")


def main():
    w = synth.WORKLOADS["fp32_L4096_shear"]
    c0 = w["c0"]
    mask = synth.bernoulli_mask(L, F, SEED)
    E = synth.load_path(w["kind"], w["steps"], synth.default_emax(w["kind"], 1.0, 1.0))[0]
    p = alm.Params(L=L, mu=1.0, lam=2.0, Y=1.0, mu0=c0 * 1.0, lam0=c0 * 2.0)
    r = alm.Solver(mask, p).step(E, fixed_iters=ITERS)
    idx = np.sort(np.random.default_rng(20240).choice(L * L, size=NSAMP, replace=False))
    y, x = np.divmod(idx, L)
    np.savez_compressed(
        OUT, L=L, f=F, seed=SEED, iters=ITERS, c0=c0, E=E, idx=idx,
        sigma=alm.voigt4(r.sigma[y, x]), eps=alm.voigt4(r.eps[y, x]), margin=r.margin[y, x],
        plastic=r.plastic[y, x], void=mask[y, x].astype(bool),
        sigma_mean=alm.voigt4(r.sigma_mean), eps_mean=alm.voigt4(r.eps_mean),
        res_eq=r.res_eq, res_mac=r.res_mac, res_cmp=r.res_cmp,
        sigma_norm=np.linalg.norm(r.sigma), plastic_count=int(r.plastic.sum()))
    print("wrote", OUT, "res_eq", r.res_eq, "res_cmp", r.res_cmp)


if __name__ == "__main__":
    main()
