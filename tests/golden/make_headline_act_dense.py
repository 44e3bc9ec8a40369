"""Writes SHA-256 digests of the oracle's input and output ciphertexts for the
activation and the dense layer of a ResNet-20-style ensemble at the ring and
chain it runs on: headline_act_dense_N65536.json.

Network: 16 channels of 32x32 in 1024-slot blocks, 4 members; a monic
quadratic activation (x^2 + b x + c per member and channel, with
relinearisation: 7 key-switching digits at the top of the tower-reuse chain,
N = 2^16, 21 Q primes, 3 P primes), then the dense layer after global sum
pooling (the slot sums by rotation, 10 classes, one plaintext per class and
channel).  Two images.

Each digest is over the ciphertext in coefficient form as little-endian
uint64 words [npoly][level+1][N].  Everything here comes from the oracle and
the seeded input generators only.  Run from the repository root:

    python tests/golden/make_headline_act_dense.py [--procs 2]
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "headline_act_dense_N65536.json")
CASE = dict(spec_seed=2018, key_seed=81, image_seed=82, images=2, C=16, M=4, classes=10, H=32, W=32, block=1024,
            stream_base=8000)
DELTA_LOG2 = 30


def digest(a) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def case_spec(c):
    from workloads.nets import act_dense_spec
    return act_dense_spec(c["spec_seed"], c["C"], c["M"], c["classes"], c["H"], c["W"], c["block"])


def _one_image(n):
    from oracle.ckks import Oracle
    from oracle.network import OracleNetwork
    from workloads import gen
    from workloads.params import resnet20_tower
    c = CASE
    ps = resnet20_tower()
    spec = case_spec(c)
    D = 2.0 ** DELTA_LOG2
    o = Oracle.from_params(ps)
    onet = OracleNetwork(o, spec, D, D, D)
    sk = o.secret_key(c["key_seed"])
    rlk = o.relin_key(sk)
    gk = {o.galois_elt(s): o.galois_key(sk, o.galois_elt(s)) for s in onet.steps()}
    imgs = gen.images(c["image_seed"], c["images"], c["C"], c["H"], c["W"])
    t0 = time.time()
    oin = onet.encrypt_image(sk, imgs[n], c["stream_base"] + n * 4096)
    oout, _ = onet.run(sk, oin, rlk, gk)
    print(f"image {n}: {time.time() - t0:.0f} s", flush=True)
    return dict(inputs=[digest(x.data) for x in oin],
                outputs=[dict(level=y.level, scale=float(y.scale).hex(), sha256=digest(y.data)) for y in oout])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=2)
    args = ap.parse_args()
    with Pool(args.procs) as pool:
        per_image = pool.map(_one_image, range(CASE["images"]))
    rec = dict(source="oracle/ (tests/golden/make_headline_act_dense.py)", params="resnet20_tower()",
               delta_log2=DELTA_LOG2, case=CASE, images=per_image)
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
