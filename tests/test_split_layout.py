"""CPU emulation of the split-column layout the GPU sweep uses for columns too
long for one workgroup: rows r = t L + c split by c-range over P parts, each
part a local DIA problem of T segments of `seg` rows (h halo rows, its own
rows, h halo rows, padding), offsets q L mapped to q seg, halo rows refreshed
from the neighbours after every Taylor term.  The emulated partitioned Taylor
action (Sec. III.B, eq. eBmpsi) must equal the single-block one, and the
block-crossing rule must reject a coupling that leaves its block.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import taylor
from workloads.circuits import transmon_cavity_system


def _layout(L, T, h, P):
    w = [L // P + (1 if q < L % P else 0) for q in range(P)]
    c0 = np.concatenate([[0], np.cumsum(w)[:-1]]).astype(int)
    seg = max(w) + 2 * h
    return w, c0, seg


def _local_dia(A, L, T, h, q, w, c0, seg, offsets):
    """Local DIA of part q: vals[e][l] for local offsets, zero on halo/padding rows."""
    d_loc = T * seg
    A = sp.csr_matrix(A)
    loc_off = [o if abs(o) <= h else (o // L) * seg for o in offsets]
    vals = np.zeros((len(offsets), d_loc), dtype=np.complex128)
    for t in range(T):
        for k in range(w[q]):
            l = t * seg + h + k
            g = t * L + c0[q] + k
            row = A.getrow(g)
            for j, v in zip(row.indices, row.data):
                vals[offsets.index(j - g), l] = v
    return vals, loc_off


def _split_action(A, psi, m, s, L, T, h, P):
    offsets = sorted(set((sp.coo_matrix(A).col - sp.coo_matrix(A).row).tolist()) | {0})
    w, c0, seg = _layout(L, T, h, P)
    d_loc = T * seg
    parts = [_local_dia(A, L, T, h, q, w, c0, seg, offsets) for q in range(P)]
    # gather the state into the local layouts (halo rows start at zero)
    loc = []
    for q in range(P):
        v = np.zeros(d_loc, dtype=np.complex128)
        for t in range(T):
            v[t * seg + h: t * seg + h + w[q]] = psi[t * L + c0[q]: t * L + c0[q] + w[q]]
        loc.append(v)

    def exchange(vecs):
        out = [v.copy() for v in vecs]
        for q in range(P):
            for t in range(T):
                for k in range(h):
                    if q > 0:   # left neighbour's last h own rows -> my low halo
                        out[q][t * seg + k] = vecs[q - 1][t * seg + w[q - 1] + k]
                    if q + 1 < P:  # right neighbour's first h own rows -> my high halo
                        out[q][t * seg + h + w[q] + k] = vecs[q + 1][t * seg + h + k]
        return out

    def apply(q, v):
        vals, loc_off = parts[q]
        out = np.zeros(d_loc, dtype=np.complex128)
        for e, lo in enumerate(loc_off):
            idx = np.arange(d_loc) + lo
            ok = (idx >= 0) & (idx < d_loc)
            out[ok] += vals[e, ok] * v[idx[ok]]
        return out

    acc = loc
    for _ in range(s):
        term = exchange(acc)          # the block is refreshed before the first term
        new_acc = [a.copy() for a in acc]
        for j in range(1, m + 1):
            term = exchange([apply(q, term[q]) / (s * j) for q in range(P)])
            new_acc = [new_acc[q] + term[q] for q in range(P)]
        # accumulators on halo rows stay those of the computed (zero-coefficient) rows
        for q in range(P):
            for t in range(T):
                new_acc[q][t * seg: t * seg + h] = 0.0
                new_acc[q][t * seg + h + w[q]: (t + 1) * seg] = 0.0
        acc = new_acc
    out = np.zeros_like(psi)
    for q in range(P):
        for t in range(T):
            out[t * L + c0[q]: t * L + c0[q] + w[q]] = acc[q][t * seg + h: t * seg + h + w[q]]
    return out


@pytest.mark.parametrize("P", [2, 3, 5])
def test_split_taylor_action_equals_single_block(P):
    d_t, d_c = 6, 40
    H0, Hk, _ = transmon_cavity_system(d_t, d_c, -2 * np.pi * 0.2, -2 * np.pi * 0.002)
    rng = np.random.default_rng(8)
    H = H0 + sum(rng.uniform(-0.3, 0.3) * h for h in Hk)
    A = -1j * 0.2 * H
    psi = rng.normal(size=d_t * d_c) + 1j * rng.normal(size=d_t * d_c)
    psi /= np.linalg.norm(psi)
    ref = taylor.taylor_action(A, psi, 12, 2)
    got = _split_action(A, psi, 12, 2, L=d_c, T=d_t, h=1, P=P)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_block_crossing_coupling_detected():
    """A short-offset entry that links two blocks (here (t, L-1) -> (t+1, 0))
    would read a halo row the split never fills: the layout rule rejects it."""
    d_t, d_c = 4, 16
    H0, Hk, _ = transmon_cavity_system(d_t, d_c, -2 * np.pi * 0.2, -2 * np.pi * 0.002)
    bad = sp.lil_matrix(H0.shape, dtype=np.complex128)
    bad[d_c - 1, d_c] = 0.1
    bad[d_c, d_c - 1] = 0.1
    M = sp.csr_matrix(H0 + bad)
    coo = sp.coo_matrix(M)
    crosses = [(i, j) for i, j in zip(coo.row, coo.col)
               if i != j and abs(j - i) <= 1 and i // d_c != j // d_c]
    assert crosses  # the library then keeps one workgroup per column or refuses
