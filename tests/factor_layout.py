"""Test helper: the tfmm_op_import host layout <-> the oracle's compressed-operator dicts.

Only used to hand the same synthetic factors to both sides (the oracle's
restoration and the library's kernels); it does no arithmetic of the method.
"""
import numpy as np

import synth


def random_factors(fmt, n, ndir, rng, ranks=None):
    """Seeded random factors for a format.  Returns (ranks_list, data (complex128 1-D), oracle_dict)."""
    n1, n2, n3 = n
    R = lambda shape, s=1.0: synth.random_complex(shape, rng, s)
    if fmt == "full":
        T = R((ndir, n1, n2, n3))
        return [], T.ravel(), {"fmt": "full", "T": T}
    if fmt == "tucker3d":
        per, rk, parts = [], [], []
        for p in range(ndir):
            r = ranks[p] if ranks is not None else tuple(int(x) for x in rng.integers(2, min(n) - 1, 3))
            C = R(r)
            Us = [R((n[i], r[i]), 1 / np.sqrt(r[i])) for i in range(3)]
            per.append((C, Us))
            rk.extend(r)
            parts += [C.ravel()] + [U.ravel() for U in Us]
        return rk, np.concatenate(parts), {"fmt": fmt, "per": per}
    if fmt == "tt3d":
        per, rk, parts = [], [], []
        for p in range(ndir):
            r1, r2 = ranks[p] if ranks is not None else tuple(int(x) for x in rng.integers(2, min(n) - 1, 2))
            U1, C, U3 = R((n1, r1), 1 / np.sqrt(r1)), R((r1, n2, r2)), R((n3, r2), 1 / np.sqrt(r2))
            per.append((U1, C, U3))
            rk.extend([r1, r2])
            parts += [U1.ravel(), C.ravel(), U3.ravel()]
        return rk, np.concatenate(parts), {"fmt": fmt, "per": per}
    if fmt == "tucker4d":
        r = ranks
        C = R(r)
        Us = [R((n[i], r[i]), 1 / np.sqrt(r[i])) for i in range(3)] + [R((ndir, r[3]), 1 / np.sqrt(r[3]))]
        return list(r), np.concatenate([C.ravel()] + [U.ravel() for U in Us]), {"fmt": fmt, "C": C, "U": Us}
    if fmt == "tt4d":
        r1, r2, r3 = ranks
        U1, C1, C2, U3 = (R((n1, r1), 1 / np.sqrt(r1)), R((r1, n2, r2), 1 / np.sqrt(r2)), R((r2, n3, r3)),
                          R((ndir, r3), 1 / np.sqrt(r3)))
        d = {"fmt": fmt, "U1": U1, "C1": C1, "C2": C2, "U3": U3}
        return list(ranks), np.concatenate([U1.ravel(), C1.ravel(), C2.ravel(), U3.ravel()]), d
    if fmt == "htucker4d":
        r1, r2, r3, r4, r12, r34 = ranks
        Us = [R((n[i], ranks[i]), 1 / np.sqrt(ranks[i])) for i in range(3)] + [R((ndir, r4), 1 / np.sqrt(r4))]
        C12, C34, B = R((r1, r2, r12), 1 / np.sqrt(r12)), R((r3, r4, r34), 1 / np.sqrt(r34)), R((r12, r34))
        d = {"fmt": fmt, "U": Us, "C12": C12, "C34": C34, "B": B}
        data = np.concatenate([U.ravel() for U in Us] + [C12.ravel(), C34.ravel(), B.ravel()])
        return list(ranks), data, d
    raise ValueError(fmt)


def oracle_to_layout(comp, n, ndir):
    """Oracle compressed dict -> (ranks, data) in the import layout."""
    fmt = comp["fmt"]
    if fmt == "full":
        return [], comp["T"].ravel()
    if fmt == "tucker3d":
        rk, parts = [], []
        for C, Us in comp["per"]:
            rk.extend(C.shape)
            parts += [C.ravel()] + [U.ravel() for U in Us]
        return rk, np.concatenate(parts)
    if fmt == "tt3d":
        rk, parts = [], []
        for U1, C, U3 in comp["per"]:
            rk.extend([C.shape[0], C.shape[2]])
            parts += [U1.ravel(), C.ravel(), U3.ravel()]
        return rk, np.concatenate(parts)
    if fmt == "tucker4d":
        return list(comp["C"].shape), np.concatenate([comp["C"].ravel()] + [U.ravel() for U in comp["U"]])
    if fmt == "tt4d":
        r = [comp["C1"].shape[0], comp["C1"].shape[2], comp["C2"].shape[2]]
        return r, np.concatenate([comp[k].ravel() for k in ("U1", "C1", "C2", "U3")])
    if fmt == "htucker4d":
        r1, r2, r12 = comp["C12"].shape
        r3, r4, r34 = comp["C34"].shape
        data = np.concatenate([U.ravel() for U in comp["U"]] + [comp["C12"].ravel(), comp["C34"].ravel(),
                                                                 comp["B"].ravel()])
        return [r1, r2, r3, r4, r12, r34], data
    raise ValueError(fmt)


def layout_to_oracle(fmt, ranks, data, n, ndir):
    """Import/export layout (ranks, complex128 data) -> the oracle's compressed-operator dict.

    The inverse of oracle_to_layout: slices and reshapes only."""
    n1, n2, n3 = n
    data = np.asarray(data, dtype=np.complex128).ravel()
    pos = [0]

    def take(shape):
        m = int(np.prod(shape))
        a = data[pos[0]:pos[0] + m].reshape(shape)
        pos[0] += m
        return a

    if fmt == "full":
        comp = {"fmt": fmt, "T": take((ndir, n1, n2, n3))}
    elif fmt == "tucker3d":
        r = np.asarray(ranks).reshape(ndir, 3)
        per = []
        for r1, r2, r3 in r:
            C = take((r1, r2, r3))
            per.append((C, [take((n1, r1)), take((n2, r2)), take((n3, r3))]))
        comp = {"fmt": fmt, "per": per}
    elif fmt == "tt3d":
        r = np.asarray(ranks).reshape(ndir, 2)
        comp = {"fmt": fmt, "per": [(take((n1, r1)), take((r1, n2, r2)), take((n3, r2))) for r1, r2 in r]}
    elif fmt == "tucker4d":
        r1, r2, r3, r4 = ranks
        C = take((r1, r2, r3, r4))
        comp = {"fmt": fmt, "C": C, "U": [take((n1, r1)), take((n2, r2)), take((n3, r3)), take((ndir, r4))]}
    elif fmt == "tt4d":
        r1, r2, r3 = ranks
        comp = {"fmt": fmt, "U1": take((n1, r1)), "C1": take((r1, n2, r2)), "C2": take((r2, n3, r3)),
                "U3": take((ndir, r3))}
    elif fmt == "htucker4d":
        r1, r2, r3, r4, r12, r34 = ranks
        Us = [take((n1, r1)), take((n2, r2)), take((n3, r3)), take((ndir, r4))]
        comp = {"fmt": fmt, "U": Us, "C12": take((r1, r2, r12)), "C34": take((r3, r4, r34)), "B": take((r12, r34))}
    else:
        raise ValueError(fmt)
    if pos[0] != data.size:
        raise ValueError(f"layout holds {data.size} entries, ranks account for {pos[0]}")
    return comp
