"""Writes c5_catalogue_reference.npz: the oracle's FP64 multipoles of one
catalogue of the large data + 5x randoms shape (10^5 clustered data points
and 5x10^5 uniform randoms, weights 1 and -N_D/N_R, a 1500 Mpc/h periodic
box, 12 radial bins over [10, 130] Mpc/h, lmax 10, every multipole with
L <= 4), too large for the oracle to run inside the GPU test suite.

Calls only the oracle (oracle/) and the seeded input generators
(paper_2408_03036_amd/catalogs.py, numpy); the GPU test regenerates the same
positions, checks their SHA-256 against the one stored here, and compares the
FP64 path's multipoles with these element by element.

    python tests/golden/make_c5_reference.py        # about 10 CPU-minutes on 8 threads
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "c5_catalogue_reference.npz")

BOX = 1500.0
EDGES = np.linspace(10.0, 130.0, 13)
LMAX, LMAX_L = 10, 4
N_DATA = 100_000
SEED = 1005


def catalogue():
    """(positions, weights, N_D) of the reference catalogue."""
    sys.path.insert(0, ROOT)
    from paper_2408_03036_amd import catalogs as C
    D = C.zeldovich(N_DATA, BOX, 5.0, 0.8, C.catalogue_seed(SEED), grid=256)
    R = C.randoms(5 * N_DATA, BOX, C.randoms_seed(SEED))
    return np.ascontiguousarray(np.vstack([D, R])), C.dr_weights(N_DATA, 5 * N_DATA), N_DATA


def digest(pos):
    return hashlib.sha256(np.ascontiguousarray(pos, dtype=np.float64).tobytes()).hexdigest()


def main():
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    pos, w, nd = catalogue()
    mults = O.all_multipoles(LMAX, LMAX_L)
    re, _, res = O.run(pos, BOX, EDGES, LMAX, mults, w=w, n_data=nd)
    np.savez_compressed(OUT, multipoles=re, mults=np.array(mults, dtype=np.int32), npairs=np.int64(res.npairs),
                        pos_sha256=np.array(digest(pos)))
    print(f"wrote {OUT}: {len(mults)} multipoles, {res.npairs} pairs")


if __name__ == "__main__":
    main()
