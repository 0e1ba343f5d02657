"""Writes the stored synthetic slices (noisy sinograms) under tests/golden/ by calling only the oracle.

    python tests/golden/make_inputs.py            # smoke_n64, plain_n128 and paper72_n128 slices
    python tests/golden/make_inputs.py --uneven   # also the 48 slices of the uneven batch
    python tests/golden/make_inputs.py --study    # also the three slices of the BOAC-vs-NAC study

Each .npz holds: meas (uint16 counts [N_a, N_b]), activity (float32 true image), geometry
(n, n_angles, n_bins, n_samples, pixel), counts, seed, stream, and the true head theta / delta_R.
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle.phantom import activity_phantom, place_disks, simulate, simulate_oversampled  # noqa: E402
import synth  # noqa: E402


def make_slice(spec: synth.SliceSpec):
    g = oracle.Geometry(spec.n, spec.n_angles, spec.n_bins, spec.n_samples, spec.pixel)
    rng_ph, rng_noise, _ = synth.streams(spec.seed, spec.stream)
    theta = synth.slice_truth(spec)
    disks = place_disks(theta[:6], synth.disk_proposals(rng_ph), synth.N_DISKS,
                        synth.DISK_R_LO, synth.DISK_R_HI)
    if spec.oversample > 1:
        meas, _, _ = simulate_oversampled(g, theta, synth.DELTA_R, disks, synth.BACKGROUND_ACTIVITY,
                                          synth.DISK_ACTIVITY, spec.counts, rng_noise, spec.oversample)
    f = activity_phantom(g, theta[:6], synth.DELTA_R, disks, synth.BACKGROUND_ACTIVITY,
                         synth.DISK_ACTIVITY)
    if spec.oversample == 1:
        meas, _ = simulate(g, theta, synth.DELTA_R, f, spec.counts, rng_noise)
    assert meas.max() < 65536
    return dict(meas=meas.astype(np.uint16), activity=f.astype(np.float32),
                geometry=np.array([spec.n, spec.n_angles, spec.n_bins, spec.n_samples]),
                pixel=np.float64(spec.pixel), counts=np.float64(spec.counts),
                seed=np.int64(spec.seed), stream=np.array(spec.stream, dtype=np.int64),
                theta=theta, delta_r=np.float64(synth.DELTA_R),
                disks=np.array(disks, dtype=np.float64), oversample=np.int64(spec.oversample))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--uneven", action="store_true")
    ap.add_argument("--study", action="store_true")
    args = ap.parse_args()
    for name in ("smoke_n64", "plain_n128"):
        spec = synth.workload(name).slices[0]
        out = os.path.join(HERE, f"slice_n{spec.n}.npz")
        np.savez_compressed(out, **make_slice(spec))
        print("wrote", out)
    spec = synth.workload("paper72_n128").slices[0]
    out = os.path.join(HERE, f"slice_n{spec.n}_a{spec.n_angles}.npz")
    np.savez_compressed(out, **make_slice(spec))
    print("wrote", out)
    if args.study:
        parts = {}
        for k, spec in enumerate(synth.study_cases()):
            for key, v in make_slice(spec).items():
                parts[f"case{k}_{key}"] = v
        out = os.path.join(HERE, "study_cases.npz")
        np.savez_compressed(out, n_cases=np.int64(len(synth.STUDY_HEADS)), **parts)
        print("wrote", out)
    if args.uneven:
        w = synth.workload("uneven48")
        parts = {}
        for s, spec in enumerate(w.slices):
            d = make_slice(spec)
            for k, v in d.items():
                parts[f"s{s:02d}_{k}"] = v
            print("slice", s, spec.n, spec.n_angles, flush=True)
        out = os.path.join(HERE, "uneven48.npz")
        np.savez_compressed(out, n_slices=np.int64(len(w.slices)), **parts)
        print("wrote", out)


if __name__ == "__main__":
    main()
