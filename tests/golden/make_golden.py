"""Write tests/golden/oracle_streams.json: digests of oracle streams on tiny
seeded fields.  Calls only the oracle (and the input generators); rerun it
only when a change to the oracle's arithmetic is justified by the paper."""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1903_07761_amd import fields  # noqa: E402

CASES = [
    # (name, generator, n, seed, block, scheme, dtype, eps fraction of range)
    ("g1_32_n8_w4_f32", "bumps", 32, 1903, 8, "W4", "float32", 1e-3),
    ("g1_32_n16_w4li_f32", "bumps", 32, 1903, 16, "W4_li", "float32", 1e-3),
    ("g1_32_n16_w3ai_f64", "bumps", 32, 1903, 16, "W3_ai", "float64", 1e-4),
    ("g2_32_n8_w3ai_f32", "bubbles", 32, 1904, 8, "W3_ai", "float32", 1e-2),
    ("g2_64_n32_w4_f64", "bubbles", 64, 1904, 32, "W4", "float64", 1e-3),
    ("g2_64_n32_w4li_f32", "bubbles", 64, 1904, 32, "W4_li", "float32", 1e-4),
]


def make_field(gen, n, seed, dtype):
    import torch

    dt = {"float32": torch.float32, "float64": torch.float64}[dtype]
    if gen == "bumps":
        return fields.gaussian_bumps(n, seed, dtype=dt).numpy()
    return fields.bubble_cloud(n, seed, nbubbles=20, dtype=dt).numpy()


def compute():
    out = {}
    for name, gen, n, seed, block, scheme, dtype, frac in CASES:
        f = make_field(gen, n, seed, dtype)
        eps = frac * float(f.max() - f.min())
        s = O.compress(f, block, scheme, eps)
        field_digest = hashlib.sha256(np.ascontiguousarray(f).tobytes()).hexdigest()
        out[name] = {"field_sha256": field_digest, "block": block, "scheme": scheme, "dtype": dtype,
                     "eps": eps, "stream_bytes": len(s), "stream_sha256": hashlib.sha256(s).hexdigest()}
    return out


if __name__ == "__main__":
    O.build(force=False)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_streams.json")
    with open(path, "w") as fh:
        json.dump(compute(), fh, indent=1, sort_keys=True)
    print("wrote", path)
