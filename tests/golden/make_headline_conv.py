"""Writes SHA-256 digests of the oracle's input and output ciphertexts for one
convolution layer of the ResNet-20-style ensemble at the ring and chain it
runs on: headline_conv_N65536.json (one plaintext per tap and centroid,
1024-slot blocks) and headline_conv_slice_N65536.json (the slice-shared
layout: one plaintext per kernel column and centroid, 2048-slot blocks whose
lower half is zero rows).

Layer: 3x3, stride 1, 16 -> 16 channels, 32x32 images, 4 members in blocks of
1024 or 2048 slots, 64 centroids per kernel column in R^4, double-hoisted (rotated
inputs in Q_l u P, one ModDown per output), at the top level of the
tower-reuse chain (N = 2^16, 21 Q primes, 3 P primes, 3 primes per digit, so
7 digits).  Four images.

Each digest is over the ciphertext in coefficient form as little-endian
uint64 words [npoly][level+1][N].  Everything here comes from the oracle and
the seeded input generators only.  Run from the repository root:

    python tests/golden/make_headline_conv.py [--procs 4] [--layout taps|slice]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = {"taps": os.path.join(HERE, "headline_conv_N65536.json"),
       "slice": os.path.join(HERE, "headline_conv_slice_N65536.json")}

CASES = {"taps": dict(spec_seed=2016, key_seed=77, image_seed=78, images=4, I=16, O=16, k=64, M=4, H=32, W=32,
                      block=1024, stream_base=6000),
         "slice": dict(spec_seed=2017, key_seed=79, image_seed=80, images=4, I=16, O=16, k=64, M=4, H=32, W=32,
                       block=2048, slice_shared=True, stream_base=7000)}
DELTA_LOG2 = 30


def digest(a) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def case_spec(c):
    from workloads.nets import single_conv_spec
    spec = single_conv_spec(c["spec_seed"], c["I"], c["O"], c["k"], c["M"], c["H"], c["W"], c["block"])
    spec["layout"]["slice_shared"] = bool(c.get("slice_shared", False))
    return spec


def _one_image(job):
    layout, n = job
    import numpy as np  # noqa: F401
    from oracle.ckks import Oracle
    from oracle.network import OracleNetwork
    from workloads import gen
    from workloads.params import resnet20_tower
    c = CASES[layout]
    ps = resnet20_tower()
    spec = case_spec(c)
    D = 2.0 ** DELTA_LOG2
    o = Oracle.from_params(ps)
    onet = OracleNetwork(o, spec, D, D, D)
    sk = o.secret_key(c["key_seed"])
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in onet.steps()}
    imgs = gen.images(c["image_seed"], c["images"], c["I"], c["H"], c["W"])
    t0 = time.time()
    oin = onet.encrypt_image(sk, imgs[n], c["stream_base"] + n * 4096)
    oout, _ = onet.run(sk, oin, rlk, gk)
    print(f"image {n}: {time.time() - t0:.0f} s", flush=True)
    return dict(inputs=[digest(x.data) for x in oin],
                outputs=[dict(level=y.level, scale=float(y.scale).hex(), sha256=digest(y.data)) for y in oout])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=4)
    ap.add_argument("--layout", default="slice", choices=sorted(CASES))
    args = ap.parse_args()
    c = CASES[args.layout]
    with Pool(args.procs) as pool:
        per_image = pool.map(_one_image, [(args.layout, n) for n in range(c["images"])])
    rec = dict(source="oracle/ (tests/golden/make_headline_conv.py)", params="resnet20_tower()",
               delta_log2=DELTA_LOG2, case=c, images=per_image)
    with open(OUT[args.layout], "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT[args.layout])


if __name__ == "__main__":
    main()
