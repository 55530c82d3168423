"""Symbolic analysis of the sparse Cholesky (host only, no GPU): the
elimination order, the fronts and the assembly tree of a host-only model
against a brute-force symbolic factorization of the period block, on
topologies with parallel lines, a hub bus, a single bus and a shared
generator bus."""
import numpy as np
import pytest

from paper_2405_14032_amd import capi, synth

import pins

CASES = {
    "tiny": lambda: synth.config_network("tiny"),
    "ragged": lambda: synth.make_network(301, 517, 63, 2, 41),
    "hub": lambda: pins.hub_network(),
    "single_period": lambda: synth.make_network(57, 80, 11, 1, 73),
    "isolated_bus": lambda: pins.manual_network(4, [0, 1], [1, 2], [0.01, 0.02], [0.1, 0.2], [0.02, 0.01], [0, 2], T=3,
                                                pd=np.full((3, 4), 0.3)),
    "one_bus": lambda: pins.manual_network(1, [], [], [], [], [], [0], T=3, pd=np.full((3, 1), 0.4)),
    "parallel": lambda: pins.manual_network(4, [0, 0, 1, 1, 2], [1, 1, 0, 2, 3], [0.01] * 5,
                                            [0.1, 0.2, 0.15, 0.1, 0.3], [0.02] * 5, [1, 1, 3], T=3,
                                            pd=np.full((3, 4), 0.2)),
}


def _period_pattern(M, net):
    """Lower pattern of period 0's diagonal block of K (local indices)."""
    rp, ci = M.kkt_structure_host()
    n_p = 2 * net.N + 2 * net.G + 4 * net.B
    rows = np.repeat(np.arange(M.n), np.diff(rp))
    keep = (rows < n_p) & (ci < n_p)
    return n_p, rows[keep], ci[keep].astype(np.int64)


def _symbolic_columns(n, rows, cols):
    """Exact column structures of the Cholesky factor of a pattern (rows >
    cols strictly lower entries), by merging each column into its parent."""
    struct = [set() for _ in range(n)]
    for r, c in zip(rows, cols):
        if r != c:
            struct[min(r, c)].add(max(r, c))
    for j in range(n):
        if struct[j]:
            par = min(struct[j])
            struct[par] |= struct[j] - {par}
    return struct


@pytest.mark.parametrize("name", list(CASES))
def test_fronts_cover_the_exact_factor(name):
    net = CASES[name]()
    M = capi.Model([net], device=-1)
    F = capi.Chol(M)
    tr = F.tree(0)
    n_p, rows, cols = _period_pattern(M, net)
    perm = tr["perm"]
    # a permutation with the pg variables last, in natural order
    assert np.array_equal(np.sort(perm), np.arange(n_p))
    n_int = n_p - net.G
    assert np.array_equal(perm[n_int:], 2 * net.N + np.arange(net.G))
    iperm = np.empty(n_p, dtype=np.int64)
    iperm[perm] = np.arange(n_p)
    struct = _symbolic_columns(n_p, iperm[rows], iperm[cols])
    first, npiv, parent, rp, rr = tr["first"], tr["npiv"], tr["parent"], tr["rowptr"], tr["rows"]
    # fronts tile the interior in order
    assert first[0] == 0 and np.array_equal(first[1:], (first + npiv)[:-1]) and first[-1] + npiv[-1] == n_int
    node_of = np.repeat(np.arange(len(first)), npiv)
    for s in range(len(first)):
        f0, f1 = first[s], first[s] + npiv[s]
        U = rr[rp[s]:rp[s + 1]]
        assert np.all(U >= f1) and np.all(np.diff(U) > 0)
        front = set(range(f0, f1)) | set(U.tolist())
        for j in range(f0, f1):
            assert struct[j] <= front, (name, s, j)
        # the parent comes later and its front holds every update row (an
        # assembly tree: with element absorption the parent need not be the
        # front of the first update row); the pg front is parent -1
        if len(U):
            if U[0] >= n_int:
                assert parent[s] == -1 and np.all(U >= n_int)
            else:
                ps = parent[s]
                assert ps > s and ps <= node_of[U[0]]
                pU = set(rr[rp[ps]:rp[ps + 1]].tolist()) | set(range(first[ps], first[ps] + npiv[ps]))
                assert set(U.tolist()) <= pU
        else:
            assert parent[s] == -1
    # the pg block: every interior column's structure reaches it only through
    # pg rows, and the dense pg front is what remains
    info = F.info()
    assert info["nodes"] == len(first)
    F.close()
    M.close()


@pytest.mark.parametrize("name", ["ragged", "paper"])
def test_amalgamation_leaves_no_near_free_merge(name):
    # merging child c into parent s adds c.p * (s.p + us - uc) explicit
    # zeros (c's rows lie in s's front); the amalgamation takes any child
    # within its 5 % budget, whatever the child's place among the parent's
    # children, so no surviving pair may cost under 0.1 % of the merged
    # front (within the pivot cap).  The rule that merged only the child
    # preceding its parent in postorder left 33 such pairs on the paper grid
    # (chains of 2-pivot fronts each passing on an update matrix of ~4500
    # rows).
    net = CASES[name]() if name in CASES else synth.make_network(10000, 13000, 2000, 2, 3)
    M = capi.Model([net], device=-1)
    F = capi.Chol(M)
    tr = F.tree(0)
    p = tr["npiv"].astype(np.int64)
    u = np.diff(tr["rowptr"]).astype(np.int64)
    par = tr["parent"]
    cheap = []
    for c in range(len(p)):
        s = par[c]
        if s < 0 or p[c] + p[s] > 4096:
            continue
        pm = p[c] + p[s]
        added = p[c] * (p[s] + u[s] - u[c])
        assert added >= 0
        if added <= 1e-3 * (pm * (pm + 1) // 2 + pm * u[s]):
            cheap.append((c, s, int(added)))
    assert not cheap, cheap[:5]
    F.close()
    M.close()


def test_fill_close_to_exact_minimum():
    # the stored factor (front blocks, explicit zeros included) stays within
    # 2x of the exact fill of the same order, and the order's fill within 2x
    # of a reverse Cuthill-McKee-free bound: the nnz of the exact factor of
    # a natural-order elimination is far larger on these grids
    net = synth.make_network(301, 517, 63, 2, 41)
    M = capi.Model([net], device=-1)
    F = capi.Chol(M)
    tr = F.tree(0)
    n_p, rows, cols = _period_pattern(M, net)
    iperm = np.empty(n_p, dtype=np.int64)
    iperm[tr["perm"]] = np.arange(n_p)
    exact = sum(len(s) for s in _symbolic_columns(n_p, iperm[rows], iperm[cols]))
    natural = sum(len(s) for s in _symbolic_columns(n_p, rows, cols))
    p = tr["npiv"].astype(np.int64)
    u = np.diff(tr["rowptr"])
    stored = int(np.sum(p * (p - 1) // 2 + p * u))
    assert exact <= stored <= 2 * exact
    assert exact * 3 < natural
    F.close()
    M.close()


def test_factor_needs_a_device():
    net = synth.config_network("tiny")
    M = capi.Model([net], device=-1)
    F = capi.Chol(M)
    with pytest.raises(ValueError, match="required"):
        F.factor(None, 0.0, 1.0, None)  # the binding refuses a missing K
    # the C ABI itself: NULL arguments / host-only model
    assert capi.opf_chol_factor(F.h, None, 0.0, 1.0, None) in (-1, -5)
    F.close()
    M.close()


def test_batched_model_one_plan_per_instance():
    nets = [synth.make_network(31, 45, 7, 3, 71), synth.make_network(14, 20, 5, 5, 72)]
    M = capi.Model(nets, device=-1)
    F = capi.Chol(M)
    t0, t1 = F.tree(0), F.tree(1)
    assert len(t0["perm"]) == 2 * 31 + 2 * 7 + 4 * 45 and len(t1["perm"]) == 2 * 14 + 2 * 5 + 4 * 20
    assert F.info()["nodes"] == len(t0["first"]) + len(t1["first"])
    F.close()
    M.close()
