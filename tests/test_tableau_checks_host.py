"""CPU checks of the torch tableau checkers (tests/tableau_checks.py) on
oracle tableaux laid out as the library lays them out (sq_layout): they pass
on valid tableaux and catch planted mistakes."""
import numpy as np
import pytest

import tableau_checks as tc
from gpu_util import mixed_program
from oracle import oracle as orc
from paper_2603_14641_amd import binding as sqb

torch = pytest.importorskip("torch")


def _to_block(n, x, z, r):
    """A uint8 torch buffer holding the oracle rows (row-major) in the
    column-major device layout of sq_layout."""
    info = sqb.layout(n)
    K, Ls = info["K"], info["Ls"]
    buf = torch.zeros(info["bytes"], dtype=torch.uint8)
    X, Z, R = tc.views(buf, info)
    bits = lambda a: np.unpackbits(a.view(np.uint8), axis=1, bitorder="little")[:, :n]  # (2n, n)
    xb, zb = bits(x), bits(z)

    def pack_cols(b):  # (2n rows, n cols) -> (n cols, 2K words)
        out = np.zeros((n, 2 * K), dtype=np.uint64)
        for half in range(2):
            rows = b[half * n:(half + 1) * n]  # (n, n)
            padded = np.zeros((K * 64, n), dtype=np.uint8)
            padded[:n] = rows
            packed = np.ascontiguousarray(np.packbits(padded.T.reshape(n, K, 64), axis=2, bitorder="little"))
            packed = packed.view(np.uint64)[:, :, 0]
            out[:, half * K:(half + 1) * K] = packed
        return out

    X[:, :2 * K] = torch.from_numpy(pack_cols(xb).view(np.int64))
    Z[:, :2 * K] = torch.from_numpy(pack_cols(zb).view(np.int64))
    rw = np.zeros(2 * K, dtype=np.uint64)
    for g in range(2 * n):
        half, i = divmod(g, n)
        if r[g]:
            rw[half * K + i // 64] |= np.uint64(1) << np.uint64(i % 64)
    R[:] = torch.from_numpy(rw.view(np.int64))
    return buf, info


@pytest.mark.parametrize("n", [1, 5, 64, 65, 130])
def test_freivalds_passes_on_oracle_tableaux_and_catches_a_flipped_bit(n):
    rng = np.random.default_rng(n)
    ops = mixed_program(rng, n, 6, p_meas=0.2)
    t = orc.Tableau(n)
    t.run(ops, seed=3)
    x, z, r = t.rows_array()
    buf, info = _to_block(n, x, z, r)
    X, Z, R = tc.views(buf, info)
    assert tc.freivalds_symplectic(X, Z, n, info["K"], probes=8, seed=1) == 0
    # a flipped x bit x_gj changes <g, h> for every h != g with z_hj = 1, so
    # the form breaks when column j of z has a 1 outside row g: some probe
    # then fails (each with probability >= 1/2)
    zb = np.unpackbits(z.view(np.uint8), axis=1, bitorder="little")[:, :n]
    cand = [(g, j) for g in range(2 * n) for j in range(n) if zb[:, j].sum() - zb[g, j] > 0]
    if not cand:
        return
    g, j = cand[int(rng.integers(len(cand)))]
    x2 = x.copy()
    x2[g, j // 64] ^= np.uint64(1) << np.uint64(j % 64)
    buf2, _ = _to_block(n, x2, z, r)
    X2, Z2, _ = tc.views(buf2, info)
    assert tc.freivalds_symplectic(X2, Z2, n, info["K"], probes=24, seed=2) > 0


@pytest.mark.parametrize("n", [3, 64, 100])
def test_basis_state_checks_after_measuring_everything(n):
    rng = np.random.default_rng(10 + n)
    ops = mixed_program(rng, n, 6, p_meas=0.0)
    meas = np.array([[orc.MEASURE, q, 0] for q in range(n)], dtype=np.uint32)
    t = orc.Tableau(n)
    bits, rnd, _ = t.run(np.concatenate([ops, meas]), seed=5)
    x, z, r = t.rows_array()
    buf, info = _to_block(n, x, z, r)
    X, Z, R = tc.views(buf, info)
    K = info["K"]
    assert tc.basis_state_stabilizers(X, Z, R, n, K, bits) == (True, True)
    single = tc.stabilizers_are_distinct_single_z(Z, n, K)
    assert single == bool(rnd.all()) or (not rnd.all())
    if rnd.all():
        assert single
    # a wrong outcome breaks the sign check; a stray x bit the x check
    wrong = bits.copy()
    wrong[int(rng.integers(n))] ^= 1
    assert tc.basis_state_stabilizers(X, Z, R, n, K, wrong)[1] is False
    x2 = x.copy()
    x2[n + int(rng.integers(n)), 0] ^= np.uint64(1)
    buf2, _ = _to_block(n, x2, z, r)
    X2, Z2, R2 = tc.views(buf2, info)
    assert tc.basis_state_stabilizers(X2, Z2, R2, n, K, bits)[0] is False


def test_single_z_check_rejects_a_product():
    n = 70
    t = orc.Tableau(n)
    meas = np.array([[orc.MEASURE, q, 0] for q in range(n)], dtype=np.uint32)
    ops = np.concatenate([np.array([[orc.H, q, 0] for q in range(n)], dtype=np.uint32), meas])
    bits, rnd, _ = t.run(ops, seed=1)
    assert rnd.all()
    x, z, r = t.rows_array()
    buf, info = _to_block(n, x, z, r)
    _, Z, _ = tc.views(buf, info)
    assert tc.stabilizers_are_distinct_single_z(Z, n, info["K"])
    z2 = z.copy()
    z2[n + 3] ^= z2[n + 4]  # S_3 <- S_3 S_4 (same group, no longer single Z's)
    buf2, _ = _to_block(n, x, z2, r)
    _, Z2, _ = tc.views(buf2, info)
    assert not tc.stabilizers_are_distinct_single_z(Z2, n, info["K"])


def test_popcount_and_parity_helpers():
    vals = np.array([0, 1, 3, 0x8000000000000000, 0xFFFFFFFFFFFFFFFF, 0x0123456789ABCDEF], dtype=np.uint64)
    t = torch.from_numpy(vals.view(np.int64))
    want = np.array([bin(int(v)).count("1") for v in vals])
    assert tc.popcount64(t).numpy().tolist() == want.tolist()
    assert tc.parity64(t).numpy().tolist() == (want % 2).tolist()
