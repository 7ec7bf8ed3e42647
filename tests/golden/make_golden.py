"""Writes oracle_regression.json: exact integer results of the FP64 oracle on
small seeded cases of every workload family and model variant.

    python tests/golden/make_golden.py

Calls only oracle/ and the seeded input generators in synth/.  The stored
values pin the oracle against unintended change (a later edit of its
arithmetic must regenerate them and say why); the GPU parity tests compare
the library with the oracle directly, not with this file.
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from synth import workloads as W  # noqa: E402

N = 20_000


def cases():
    yield "tiny", W.tiny(n_histories=N)
    yield "water_cbct_s8", W.water_cbct(scale=8, n_histories=N)
    yield "head_s8", W.head(scale=8, n_histories=N)
    wh = W.head(scale=8, n_histories=N)
    wh.compton = "wh"
    yield "head_s8_bound_compton", wh
    yield "head_helical_s8", W.head_helical(scale=8, n_histories=N)
    yield "water_box_bowtie_s5", W.water_box_bowtie(scale=5, n_histories=N)
    mh = W.water_box_bowtie(scale=5, n_histories=N)
    mh.geometry["fluence_chains"] = 256
    yield "water_box_bowtie_s5_mh", mh


def summarise(wl):
    r = O.run(O.OracleCase(wl), threads=4)
    s1 = np.ascontiguousarray(r["s1"], dtype=np.int64)
    return dict(n_histories=int(wl.n_histories), q_dep=str(int(r["q_dep"])),
                q_esc=str(int(r["q_esc"])), q_inc=str(int(r["q_inc"])),
                n_steps=int(r["n_steps"]), n_pe=int(r["n_pe"]),
                n_compton=int(r["n_compton"]), n_rayleigh=int(r["n_rayleigh"]),
                n_escapes=int(r["n_escapes"]), n_miss=int(r["n_miss"]),
                s1_sha256=hashlib.sha256(s1.tobytes()).hexdigest())


def main():
    out = {name: summarise(wl) for name, wl in cases()}
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
