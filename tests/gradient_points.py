"""Flux points whose gradient the common flux reads (LDG, beta = 1/2): side L
of every interface pair and every boundary point, per element type as
[E][N_f] booleans, from the oracle's pairing (side L sorts first by
type-major element id and local face, as in the library)."""
import numpy as np


def read_points(O):
    mark = np.zeros(O.nfpts_total, bool)
    mark[O.pair_L] = True
    if O.bnd_idx is not None and len(O.bnd_idx):
        mark[O.bnd_idx] = True
    out = {}
    for n, tg in O.types.items():
        o = O.fpt_offset[n]
        out[n] = mark[o:o + tg.nelem * tg.ref.nfpts].reshape(tg.nelem, tg.ref.nfpts)
    return out
