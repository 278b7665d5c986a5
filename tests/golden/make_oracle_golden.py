"""Writes oracle_config0.json: the FP64 oracle's round trip of the
1x9x64x64 clip (pixel seed 0, weight seed 1).  Calls only the oracle and
the seeded input generator."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import tokenizer as O  # noqa: E402


def main():
    u8 = synth.make_batch([0], 9, 64, 64)
    w = synth.make_weights(1)
    r = O.roundtrip(u8, {k: v.astype(np.float64) for k, v in w.items()})
    out = dict(
        note="FP64 oracle round trip, clip 1x9x64x64 seed 0, He-normal weights seed 1, no drop",
        clip_sha256=synth.sha256(u8),
        weights_sha256=synth.sha256(synth.flatten_weights(w)),
        idx=r["idx"].reshape(-1).tolist(),
        xhat_every_97th=r["xhat"].reshape(-1)[::97].tolist(),
        xhat_std=float(r["xhat"].std()),
        z_std=float(r["z"].std()),
    )
    with open(os.path.join(HERE, "oracle_config0.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
