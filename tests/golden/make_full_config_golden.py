"""Write the oracle's expected values for the full-size GPU parity tests.

    python tests/golden/make_full_config_golden.py [c2 c3 c5]

Calls only the FP64 oracle (oracle/) on inputs from the seeded generator
(fcgen); nothing here touches the GPU library.  Per configuration it stores,
for a sample of universes (indices into the configuration's universe array),
Algorithm 1's outputs (Delta chi^2, chi^2 minimum, argmin, chi^2 at the true
point, second-best chi^2 at another grid point), and for the true points whose
universes are all in the sample the critical values at 0.6827 / 0.90 / 0.95
and the 200-bin histogram on [0, 50) (Section 1, Figure 1), plus a fingerprint
of the inputs so that a changed generator is detected rather than compared.

  c2: all 2000 universes of 4 of the 256 true points; critical values and
      histograms of all 256 true points (the oracle runs on every universe)
  c3: the first 64 universes of each of the 64 true points, plus all 4000
      universes of 2 true points (full-K critical values)
  c5: the first 16 universes of each of the 16 true points
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import fcgen  # noqa: E402
import oracle  # noqa: E402

ALPHA = (0.6827, 0.9, 0.95)
FULL_POINTS = {"c2": (0, 85, 170, 255), "c3": (0, 63), "c5": ()}
FIRST = {"c2": 0, "c3": 64, "c5": 16}
# configurations whose every universe goes through the oracle, for the
# critical values of every true point
EVERY_POINT = ("c2",)


def fingerprint(pr, idx) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pr.S).tobytes())
    h.update(np.ascontiguousarray(pr.F).tobytes())
    h.update(np.ascontiguousarray(pr.d[idx]).tobytes())
    h.update(np.ascontiguousarray(pr.p_idx[idx]).tobytes())
    return h.hexdigest()


def sample(pr, name):
    idx = set()
    for s in range(len(pr.seg_off) - 1):
        lo, hi = int(pr.seg_off[s]), int(pr.seg_off[s + 1])
        idx.update(range(lo, min(hi, lo + FIRST[name])))
        if s in FULL_POINTS[name]:
            idx.update(range(lo, hi))
    return np.array(sorted(idx), dtype=np.int64)


def path(name):
    return os.path.join(HERE, f"{name}_oracle.npz")


def make(name):
    t0 = time.time()
    pr = fcgen.make_problem(name)
    idx = sample(pr, name)
    extra = {}
    if name in EVERY_POINT:
        every = oracle.scan(pr.S, pr.F, pr.d, pr.p_idx)
        ref = {k: v[idx] for k, v in every.items()}
        extra["crit_all"], extra["hist_all"] = oracle.critical_value(
            every["dchi2"], np.asarray(pr.seg_off, dtype=np.int64), ALPHA)
        extra["input_fingerprint_all"] = np.array(fingerprint(pr, np.arange(pr.K)))
    else:
        ref = oracle.scan(pr.S, pr.F, pr.d[idx], pr.p_idx[idx])
    full = np.array(FULL_POINTS[name], dtype=np.int64)
    seg = []
    for s in full:
        lo, hi = int(pr.seg_off[s]), int(pr.seg_off[s + 1])
        pos = np.searchsorted(idx, np.arange(lo, hi))
        assert np.array_equal(idx[pos], np.arange(lo, hi))
        seg.append(ref["dchi2"][pos])
    if seg:
        off = np.concatenate([[0], np.cumsum([len(x) for x in seg])]).astype(np.int64)
        crit, hist = oracle.critical_value(np.concatenate(seg), off, ALPHA)
    else:
        crit = np.zeros((0, len(ALPHA)))
        hist = np.zeros((0, 201), dtype=np.int64)
    np.savez_compressed(path(name), idx=idx, fingerprint=np.array(fingerprint(pr, idx)),
                        full_points=full, alpha=np.array(ALPHA), crit=crit, hist=hist,
                        **extra,
                        **{k: ref[k] for k in ("dchi2", "chi2_min", "argmin", "chi2_p",
                                               "chi2_2nd")})
    print(f"{name}: {idx.shape[0]} universes x {pr.G} grid points in {time.time() - t0:.0f} s "
          f"-> {path(name)}", flush=True)


def load(name, pr=None):
    """The stored values (dict); with ``pr`` the input fingerprint is checked."""
    z = np.load(path(name), allow_pickle=False)
    out = {k: z[k] for k in z.files}
    if pr is not None and ("input_fingerprint_all" in out and
                           str(out["input_fingerprint_all"]) != fingerprint(pr, np.arange(pr.K))):
        raise RuntimeError(f"{name}: the generator's inputs changed since the expected "
                           "values were written; run this script again")
    if pr is not None and str(out["fingerprint"]) != fingerprint(pr, out["idx"]):
        raise RuntimeError(f"{name}: the generator's inputs changed since the expected "
                           "values were written; run this script again")
    return out


if __name__ == "__main__":
    for n in (sys.argv[1:] or ["c2", "c3", "c5"]):
        make(n)
