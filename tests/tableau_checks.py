"""Invariant checks of a tableau held in a torch device buffer (sq_create_in),
computed with plain torch integer ops on the GPU. Test infrastructure: these
read the tableau's bits through the layout sq_layout reports and share no
code with the HIP kernels or the oracle.

What they check (the paper's "Measurements in the Stabilizer Formalism" and
"The CHP algorithm"; the symplectic structure of the destabilizer tableau):
  * symplectic form: for rows g, h the product <g, h> = x_g . z_h + z_g . x_h
    (mod 2) equals 1 exactly for the pairs (D_i, S_i), 0 otherwise. Checked
    with Freivalds probes: for a random row vector v, Omega v = J v, where
    Omega is the matrix of <., .> and J swaps the destabilizer and stabilizer
    halves. A wrong Omega passes one probe with probability at most 1/2;
  * after every qubit has been measured the state is the basis state |b>
    with b the outcomes, so every stabilizer is a Z string Z^z with sign
    r = z . b (mod 2): x = 0 in the whole stabilizer half and the sign bits
    equal those parities;
  * when every measurement was random, each stabilizer is exactly one +-Z_q
    and the q are distinct: the stabilizer half of Z is a permutation matrix.
"""
from __future__ import annotations

import numpy as np


def views(buf, info):
    """(X, Z, R) int64 views of a tableau block: X, Z of shape (n, Ls), R of (L,)."""
    import torch
    n, Ls, L = info["n"], info["Ls"], info["L"]
    words = buf.view(torch.int64)
    x0, z0, r0 = info["x_offset"] // 8, info["z_offset"] // 8, info["r_offset"] // 8
    X = words[x0:x0 + n * Ls].view(n, Ls)
    Z = words[z0:z0 + n * Ls].view(n, Ls)
    R = words[r0:r0 + L]
    return X, Z, R


def parity64(t):
    """Bit 0 of the result = parity of each int64 word (arithmetic shifts only
    disturb the high bits, which the fold never moves down)."""
    for s in (32, 16, 8, 4, 2, 1):
        t = t ^ (t >> s)
    return t & 1


def popcount64(t):
    """Number of set bits of each int64 word (SWAR; two's-complement wrap)."""
    import torch
    m1 = torch.tensor(0x5555555555555555, dtype=torch.int64, device=t.device)
    m2 = torch.tensor(0x3333333333333333, dtype=torch.int64, device=t.device)
    m4 = torch.tensor(0x0F0F0F0F0F0F0F0F, dtype=torch.int64, device=t.device)
    h = torch.tensor(0x0101010101010101, dtype=torch.int64, device=t.device)
    t = t - ((t >> 1) & m1)
    t = (t & m2) + ((t >> 2) & m2)
    t = (t + (t >> 4)) & m4
    return (t * h) >> 56


def xor_reduce(t, dim):
    """XOR of all slices of t along dim (a halving tree)."""
    import torch
    if t.shape[dim] == 0:
        shape = list(t.shape)
        shape[dim] = 1
        return torch.zeros(shape, dtype=t.dtype, device=t.device).squeeze(dim)
    while t.shape[dim] > 1:
        m = t.shape[dim]
        h = m // 2
        a = t.narrow(dim, 0, h) ^ t.narrow(dim, h, h)
        if m % 2:
            a = torch.cat([a, t.narrow(dim, 2 * h, 1)], dim)
        t = a
    return t.squeeze(dim)


def or_reduce(t, dim):
    import torch
    while t.shape[dim] > 1:
        m = t.shape[dim]
        h = m // 2
        a = t.narrow(dim, 0, h) | t.narrow(dim, h, h)
        if m % 2:
            a = torch.cat([a, t.narrow(dim, 2 * h, 1)], dim)
        t = a
    return t.squeeze(dim)


def row_mask_words(n, K, device):
    """int64 words (L = 2K) with the bits of rows < n set in each half."""
    import torch
    m = np.full(K, -1, dtype=np.int64)
    if n % 64:
        m[K - 1] = np.int64((1 << (n % 64)) - 1)
    half = torch.tensor(m, device=device)
    return torch.cat([half, half])


def _selected_xor(M, sel, L, chunk):
    """XOR over the columns j with sel[j] of M[j, :L]."""
    import torch
    acc = torch.zeros(L, dtype=torch.int64, device=M.device)
    idx = torch.nonzero(sel).flatten()
    for a in range(0, idx.numel(), chunk):
        acc ^= xor_reduce(M[idx[a:a + chunk], :L], 0)
    return acc


def freivalds_symplectic(X, Z, n, K, probes=4, seed=0, chunk=8192):
    """Number of failed probes of Omega v = J v (0 means every probe passed)."""
    import torch
    L = 2 * K
    dev = X.device
    rng = np.random.default_rng(seed)
    mask = row_mask_words(n, K, dev)
    fails = 0
    for _ in range(probes):
        v = torch.from_numpy(rng.integers(0, 1 << 64, L, dtype=np.uint64).view(np.int64)).to(dev) & mask
        # a_j = z_j . v, b_j = x_j . v (per column j, over all 2n rows)
        a = torch.empty(n, dtype=torch.int64, device=dev)
        b = torch.empty(n, dtype=torch.int64, device=dev)
        for j0 in range(0, n, chunk):
            j1 = min(n, j0 + chunk)
            a[j0:j1] = parity64(xor_reduce(Z[j0:j1, :L] & v, 1))
            b[j0:j1] = parity64(xor_reduce(X[j0:j1, :L] & v, 1))
        # (Omega v)_g = x_g . a + z_g . b
        om = _selected_xor(X, a != 0, L, chunk) ^ _selected_xor(Z, b != 0, L, chunk)
        jv = torch.cat([v[K:L], v[:K]])
        if not torch.equal(om, jv):
            fails += 1
    return fails


def basis_state_stabilizers(X, Z, R, n, K, bits):
    """After every qubit was measured with outcomes `bits` (uint8 per qubit):
    (stabilizer x bits all zero, stabilizer signs equal z . b for every row)."""
    import torch
    L = 2 * K
    dev = X.device
    x_zero = not bool(torch.any(X[:, K:L] != 0).item())
    b = torch.as_tensor(np.asarray(bits, dtype=np.uint8), device=dev) != 0
    par = _selected_xor(Z, b, L, 8192)[K:L]
    mask = row_mask_words(n, K, dev)[K:L]
    signs_ok = torch.equal(par & mask, R[K:L] & mask)
    return x_zero, signs_ok


def stabilizers_are_distinct_single_z(Z, n, K):
    """Whether the stabilizer half of Z is a permutation matrix (every S_i a
    single Z_q, every q once)."""
    import torch
    L = 2 * K
    S = Z[:, K:L]
    per_col = popcount64(S).sum(1)
    if not bool(torch.all(per_col == 1).item()):
        return False
    covered = or_reduce(S, 0)
    mask = row_mask_words(n, K, Z.device)[K:L]
    return torch.equal(covered, mask)
