"""Write ``nep_synth/model_scales.json`` from the FP64 oracle (test infrastructure).

The random model's descriptor scale is s_nu = 1 / RMS(q_nu) over the atoms
of the tiny workload (2,000-atom bcc W, sigma = 0.05 A), so that scaled
descriptors are of order one and the tanh layer is not saturated.  The
output weights are then multiplied by kappa, chosen so that the RMS force
of the network part on that workload is 1 eV/A; the sign of kappa makes the
lattice restoring on average (sum_i F_i . u_i < 0 for the displacements
u_i from the lattice sites of atoms that are not in a ZBL pair).

Both the default model and the paper-size one (nep_synth.PAPER_DIMS) are
calibrated; the latter under the key "paper".

Usage:  python -m oracle.calibrate
"""
from __future__ import annotations

import json

import numpy as np

import nep_synth
import oracle


def calibrate(size="small"):
    m = nep_synth.random_model(scaled=False, size=size)
    m.zbl_r2 = m.zbl_r1 = 0.0   # network part only
    sysm = nep_synth.tiny()
    pos, h = sysm.pos, sysm.h[0]
    r = oracle.efv_cell(m, pos, h, desc=True, virial=False)
    q = r["desc"]
    rms = np.sqrt(np.mean(q * q, axis=0))
    m.q_scale = 1.0 / rms
    r = oracle.efv_cell(m, pos, h, virial=False)
    F = r["forces"]
    lattice, _ = nep_synth.bcc_lattice(10, 10, 10)
    disp = pos - lattice
    mask = np.ones(pos.shape[0], bool)
    for i, j, _ in sysm.meta["pulled_pairs"]:
        mask[i] = mask[j] = False
    restoring = float(np.sum(F[mask] * disp[mask]))
    kappa = 1.0 / float(np.sqrt(np.mean(np.sum(F[mask] ** 2, axis=1))))
    if restoring > 0.0:
        kappa = -kappa
    return {"q_scale": (1.0 / rms).tolist(), "kappa": kappa,
            "note": "q_scale = 1/RMS descriptor and kappa = output-weight factor, "
                    "from the FP64 oracle on the tiny workload (oracle/calibrate.py)"}


if __name__ == "__main__":
    out = calibrate()
    out["paper"] = calibrate("paper")
    with open(nep_synth.SCALES_PATH, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
