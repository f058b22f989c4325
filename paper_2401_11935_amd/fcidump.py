"""Real-integral ingestion: FCIDUMP reader and writer, pivoted Cholesky
factorisation of the two-electron integrals into the factors B[P, p, q] that
the library takes, and the spin-averaged Fock matrix F.

The library's Hamiltonian is (pq|rs) = sum_P B[P,p,q] B[P,r,s] with a
one-electron part h = F - G_avg[B] (the spin-averaged open-shell Fock matrix
F, with G_avg as in `spin_averaged_fock` below); orbitals are ordered
[core | t | u | virtuals].  An FCIDUMP gives h and (pq|rs) in its own orbital
order; `load_problem` reorders them, factorises the integrals and forms F.

Supported FCIDUMP content: one set of real spatial integrals (the RHF/ROHF
form) in chemists' notation with 1-based indices, eight-fold permutational
symmetry, one-electron lines "x i j 0 0", the core energy "x 0 0 0 0".
Spin-blocked (UHF) files are not supported.  The integrals are held as a
dense n^2 x n^2 matrix, which bounds n by host memory (n = 150: 4 GB).

Host-side NumPy; nothing here runs on the device.
"""
from __future__ import annotations

import re

import numpy as np


def read_fcidump(path: str) -> dict:
    """Parses an FCIDUMP file: {"norb", "nelec", "ms2", "h" (n x n), "eri"
    (n, n, n, n) with all eight permutations filled, "e_core"}."""
    with open(path) as f:
        text = f.read()
    m = re.search(r"(&END|/)\s*\n", text, flags=re.IGNORECASE)
    if not m or not text.lstrip().upper().startswith("&FCI"):
        raise ValueError("not an FCIDUMP file: no &FCI ... &END header")
    header, body = text[:m.start()], text[m.end():]

    def field(name, default=None):
        mm = re.search(name + r"\s*=\s*(-?\d+)", header, flags=re.IGNORECASE)
        if mm is None:
            if default is None:
                raise ValueError(f"FCIDUMP header has no {name}")
            return default
        return int(mm.group(1))

    n = field("NORB")
    nelec = field("NELEC", 0)
    ms2 = field("MS2", 0)
    rows = [ln.split() for ln in body.replace("D", "E").replace("d", "e").splitlines() if ln.strip()]
    if any(len(r) != 5 for r in rows):
        raise ValueError("FCIDUMP integral lines must hold a value and four indices")
    val = np.array([float(r[0]) for r in rows])
    idx = np.array([[int(x) for x in r[1:]] for r in rows], dtype=np.int64)
    if idx.size and (idx.min() < 0 or idx.max() > n):
        raise ValueError("FCIDUMP orbital index out of range")
    h = np.zeros((n, n))
    eri = np.zeros((n, n, n, n))
    e_core = 0.0
    for x, (i, j, k, l) in zip(val, idx):
        if i and j and k and l:
            i, j, k, l = i - 1, j - 1, k - 1, l - 1
            for (a, b, c, d) in ((i, j, k, l), (j, i, k, l), (i, j, l, k), (j, i, l, k),
                                 (k, l, i, j), (l, k, i, j), (k, l, j, i), (l, k, j, i)):
                eri[a, b, c, d] = x
        elif i and j and not k and not l:
            h[i - 1, j - 1] = h[j - 1, i - 1] = x
        elif not (i or j or k or l):
            e_core = x
        else:
            raise ValueError(f"unsupported FCIDUMP index pattern {(i, j, k, l)}")
    return {"norb": n, "nelec": nelec, "ms2": ms2, "h": h, "eri": eri, "e_core": e_core}


def write_fcidump(path: str, h: np.ndarray, eri: np.ndarray, nelec: int, ms2: int = 0, e_core: float = 0.0,
                  tol: float = 0.0) -> None:
    """Writes h and (pq|rs) (eight-fold unique entries with |x| > tol) as an FCIDUMP file."""
    n = h.shape[0]
    lines = [f"&FCI NORB={n},NELEC={nelec},MS2={ms2},", " ORBSYM=" + "1," * n, " ISYM=1,", "&END"]
    for i in range(n):
        for j in range(i + 1):
            ij = i * (i + 1) // 2 + j
            for k in range(n):
                for l in range(k + 1):
                    if k * (k + 1) // 2 + l > ij:
                        continue
                    x = eri[i, j, k, l]
                    if abs(x) > tol:
                        lines.append(f"{x:.17e} {i + 1} {j + 1} {k + 1} {l + 1}")
    for i in range(n):
        for j in range(i + 1):
            if abs(h[i, j]) > tol:
                lines.append(f"{h[i, j]:.17e} {i + 1} {j + 1} 0 0")
    lines.append(f"{e_core:.17e} 0 0 0 0")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def pivoted_cholesky(eri: np.ndarray, tol: float = 1e-10, max_rank: int | None = None) -> np.ndarray:
    """Factors B[P, p, q] with sum_P B[P,p,q] B[P,r,s] = (pq|rs) to within tol
    on the diagonal of the remainder: pivoted (incomplete) Cholesky of the
    positive semi-definite matrix V[(pq), (rs)] = (pq|rs), choosing at each step
    the largest remaining diagonal element (Beebe-Linderberg)."""
    n = eri.shape[0]
    V = eri.reshape(n * n, n * n)
    d = np.array(np.diag(V), dtype=np.float64)
    if d.min() < -1e-10:
        raise ValueError("two-electron integrals are not positive semi-definite")
    cap = n * n if max_rank is None else max_rank
    L = []
    while len(L) < cap:
        p = int(np.argmax(d))
        if d[p] <= tol:
            break
        col = np.array(V[:, p], dtype=np.float64)
        for l in L:
            col -= l * l[p]
        if col[p] <= tol:
            break
        l = col / np.sqrt(col[p])
        L.append(l)
        d -= l * l
    B = np.array(L).reshape(len(L), n, n)
    return 0.5 * (B + B.transpose(0, 2, 1))


def g_avg(B: np.ndarray, nc: int) -> np.ndarray:
    """G_avg,pq = sum_{k in core} [2 (pq|kk) - (pk|kq)] + sum_{x in {t,u}} [(pq|xx) - 1/2 (px|xq)],
    with t = nc, u = nc + 1."""
    occ = np.arange(nc)
    act = np.array([nc, nc + 1])
    J = lambda ks: np.einsum("Ppq,Pkk->pq", B, B[:, ks][:, :, ks])  # noqa: E731
    K = lambda ks: np.einsum("Ppk,Pkq->pq", B[:, :, ks], B[:, ks, :])  # noqa: E731
    return 2.0 * J(occ) - K(occ) + J(act) - 0.5 * K(act)


def spin_averaged_fock(h: np.ndarray, B: np.ndarray, nc: int) -> np.ndarray:
    """F = h + G_avg[B]: the spin-averaged Fock matrix of the open-shell reference
    (the inverse of the library's h = F - G_avg[B])."""
    return h + g_avg(B, nc)


def reorder(h: np.ndarray, eri: np.ndarray, order) -> tuple[np.ndarray, np.ndarray]:
    """h and (pq|rs) with orbital i of the result = orbital order[i] of the input."""
    o = np.asarray(order, dtype=np.int64)
    if sorted(o.tolist()) != list(range(h.shape[0])):
        raise ValueError("order must be a permutation of the orbitals")
    return h[np.ix_(o, o)], eri[np.ix_(o, o, o, o)]


def load_problem(path: str, core, t: int, u: int, virt=None, tol: float = 1e-10) -> dict:
    """Reads an FCIDUMP and returns the library's inputs for an open-shell
    problem: B (naux, n, n) and F (n, n) in the order [core | t | u | virt],
    nc, nv, naux, and the FCIDUMP's core energy.  core and virt are 0-based
    orbital indices of the file (virt defaults to all remaining orbitals in
    file order); t and u are the singly occupied orbitals."""
    d = read_fcidump(path)
    n = d["norb"]
    core = [int(x) for x in core]
    if virt is None:
        taken = set(core) | {t, u}
        virt = [i for i in range(n) if i not in taken]
    order = core + [t, u] + [int(x) for x in virt]
    h, eri = reorder(d["h"], d["eri"], order)
    B = pivoted_cholesky(eri, tol=tol)
    nc = len(core)
    F = spin_averaged_fock(h, B, nc)
    return {"B": np.ascontiguousarray(B), "F": F, "nc": nc, "nv": n - nc - 2, "naux": B.shape[0],
            "e_core": d["e_core"], "nelec": d["nelec"], "ms2": d["ms2"]}
