#!/usr/bin/env python
"""Writes the stored oracle results the large GPU parity tests compare with.

Every expected value here comes from the CPU oracle (``oracle/``, the direct
sums of the synthesis of Sec. I, eq. syn, and of its adjoint) evaluated on
seeded inputs from ``paper_2603_17166_amd.synthetic`` (which holds no
arithmetic of the method).  Nothing is taken from the GPU library.

Fixtures (numpy .npz, loadable with allow_pickle=False):

* ``spt1501_l4096_s2.npz`` -- the 1501 deg^2, 0.5', lmax 4096, spin-2 patch
  (21.6 M points; the same points and coefficients serve its FP32 eps 1e-5 and
  FP64 eps 1e-10 plans):
    - ``idx``: the seeded 10 000-point subsample (Workload.subsample, seed
      4003), with ``theta``/``phi`` at those points (reproduction check);
    - ``synth``: the oracle synthesis of the workload's coefficients
      (seed 1003) at those points;
    - ``adj_in``: complex64 map values on the subsample (seed 3503); the map
      is zero everywhere else;
    - ``adj_k``: a seeded set (seed 4503) of 20 480 coefficient indices, and
      ``adj_out`` (2, 20480): the oracle adjoint of that map at those indices.
* ``served_discs.npz`` -- for every disc of the served mix (radius 2, 5, 10,
  20 deg), lmax 512 .. 4096 and spin 0 / 2, keys ``r{R}_l{L}_s{S}_*``: a
  64-point synthesis check (coefficient seed 5000 + code, subsample seed
  5100 + code) and an adjoint check from a complex64 map on 64 points (seed
  5200 + code) stored on 2048 seeded coefficients (seed 5300 + code), where
  code = 100 R + L / 512 + S.

A sidecar ``fixtures.json`` records the seeds and the SHA-256 of this script
and of ``oracle/oracle.c`` at generation time.

Usage: ``python tests/golden/make_fixtures.py [spt|served|all]`` (about
25 min for the lmax 4096 patch on 8 cores, 3 min for the discs).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2603_17166_amd import synthetic as syn  # noqa: E402

SPT_FILE = os.path.join(HERE, "spt1501_l4096_s2.npz")
SERVED_FILE = os.path.join(HERE, "served_discs.npz")
META_FILE = os.path.join(HERE, "fixtures.json")

SPT_SUB = 10000
SPT_ADJ_SEED = 3503
SPT_K_SEED = 4503
SPT_NK = 20480

DISC_NPTS = 64
DISC_NK = 2048


def _sha(path: str) -> str:
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def disc_code(radius: float, lmax: int, spin: int) -> int:
    return int(100 * radius) + lmax // 512 + spin


def log(msg: str) -> None:
    print("[fixtures] " + msg, flush=True)


def make_spt() -> dict:
    w = syn.spt_fine("fp64")
    idx = w.subsample(SPT_SUB)
    th, ph = w.theta[idx], w.phi[idx]
    a = w.alm()
    t0 = time.time()
    f = np.empty(idx.shape[0], dtype=np.complex128)
    for c in range(0, idx.shape[0], 1000):
        f[c:c + 1000] = oracle.synth(a, th[c:c + 1000], ph[c:c + 1000], w.lmax, w.spin)
        log("spt synth %d / %d points (%.0f s)" % (min(c + 1000, idx.shape[0]), idx.shape[0], time.time() - t0))
    g = syn.gaussian_map(idx.shape[0], SPT_ADJ_SEED, np.complex64)
    t0 = time.time()
    at = oracle.adjoint(g.astype(np.complex128), th, ph, w.lmax, w.spin)
    log("spt adjoint (%.0f s)" % (time.time() - t0))
    k = np.sort(syn.rng(SPT_K_SEED).choice(syn.nalm(w.lmax), size=SPT_NK, replace=False))
    np.savez(SPT_FILE, idx=idx, theta=th, phi=ph, synth=f, adj_in=g, adj_k=k, adj_out=at[:, k])
    return {"workload": w.name[:-5], "npoints": w.npoints, "lmax": w.lmax, "spin": w.spin,
            "seeds": {"points": syn.SEED_POINTS + 3, "alm": syn.SEED_ALM + 3, "subsample": syn.SEED_SUBSAMPLE + 3,
                      "adjoint_map": SPT_ADJ_SEED, "coefficient_subset": SPT_K_SEED},
            "subsample": SPT_SUB, "coefficients_stored": SPT_NK}


def make_served() -> dict:
    out = {}
    t0 = time.time()
    for r in syn.SERVED_RADII:
        th_all, ph_all = syn.served_patch(r)
        for lmax in syn.SERVED_LMAX:
            for spin in syn.SERVED_SPINS:
                code = disc_code(r, lmax, spin)
                pre = "r%g_l%d_s%d_" % (r, lmax, spin)
                a = syn.gaussian_alm(lmax, spin, 5000 + code)
                idx = np.sort(syn.rng(5100 + code).choice(th_all.shape[0], size=DISC_NPTS, replace=False))
                out[pre + "idx"] = idx.astype(np.int32)
                out[pre + "synth"] = oracle.synth(a, th_all[idx], ph_all[idx], lmax, spin)
                g = syn.gaussian_map(DISC_NPTS, 5200 + code, np.complex64)
                at = oracle.adjoint(g.astype(np.complex128), th_all[idx], ph_all[idx], lmax, spin)
                k = np.sort(syn.rng(5300 + code).choice(syn.nalm(lmax), size=min(DISC_NK, syn.nalm(lmax)),
                                                        replace=False))
                out[pre + "adj_in"] = g
                out[pre + "adj_k"] = k.astype(np.int32)
                out[pre + "adj_out"] = at[:, k]
                log("disc %g deg lmax %d spin %d (%.0f s)" % (r, lmax, spin, time.time() - t0))
    np.savez(SERVED_FILE, **out)
    return {"radii": list(syn.SERVED_RADII), "lmax": list(syn.SERVED_LMAX), "spins": list(syn.SERVED_SPINS),
            "npoints_checked": DISC_NPTS, "coefficients_stored": DISC_NK,
            "seeds": "alm 5000 + code, subsample 5100 + code, map 5200 + code, coefficients 5300 + code; "
                     "code = 100 radius + lmax / 512 + spin"}


def main() -> int:
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    oracle.build(force=False)
    meta = {}
    if os.path.exists(META_FILE):
        with open(META_FILE) as fh:
            meta = json.load(fh)
    stamp = {"script_sha256": _sha(os.path.abspath(__file__)),
             "oracle_c_sha256": _sha(os.path.join(ROOT, "oracle", "oracle.c"))}
    if which in ("spt", "all"):
        meta["spt1501_l4096_s2.npz"] = dict(make_spt(), **stamp)
    if which in ("served", "all"):
        meta["served_discs.npz"] = dict(make_served(), **stamp)
    with open(META_FILE, "w") as fh:
        json.dump(meta, fh, indent=1, sort_keys=True)
        fh.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
