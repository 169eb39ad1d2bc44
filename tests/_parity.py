"""Parity checks between the GPU library and the FP64 oracle.

Tolerances (written here, used by every GPU test):
* accumulator entries: |gpu - ref| <= 1e-5 |ref| + amb + 1e-12, where amb is
  the oracle's ambiguity mass (exact weight change of marginal 3DGS decisions);
* contribution count: |gpu - ref| <= the oracle's count slack;
* Top-K indices: equal except where the values that decide them lie within
  the entry tolerance of each other (near ties, including the K-th/K+1-th
  boundary); order checked wherever adjacent values are separated by more;
* Top-K values: normalised by the GPU's own chosen set, 1e-5 relative.
"""
import numpy as np

ACC_REL = 1e-5
ACC_ABS = 1e-12


def check_acc(gpu_acc: np.ndarray, ref_acc: np.ndarray, amb: np.ndarray, rel=ACC_REL):
    gpu_acc = np.asarray(gpu_acc, np.float64)
    err = np.abs(gpu_acc - ref_acc)
    tol = rel * np.abs(ref_acc) + amb + ACC_ABS
    bad = err > tol
    n_amb = int(((err > rel * np.abs(ref_acc) + ACC_ABS) & ~bad).sum())
    nz = ref_acc != 0
    stats = dict(max_rel=float((err[nz] / np.abs(ref_acc[nz])).max()) if nz.any() else 0.0,
                 n_bad=int(bad.sum()), n_needed_amb=n_amb, n_entries=int(nz.sum()))
    if bad.any():
        i, j = np.argwhere(bad)[0]
        raise AssertionError(f"acc mismatch at ({i},{j}): gpu={gpu_acc[i, j]!r} ref={ref_acc[i, j]!r} "
                             f"amb={amb[i, j]!r}; {stats}")
    return stats


def check_topk(gpu_idx: np.ndarray, gpu_val: np.ndarray, ref_acc: np.ndarray, amb: np.ndarray,
               k: int, rel=ACC_REL):
    """Index sets/orders and values of the GPU Top-K against the FP64 accumulator."""
    ref_acc = np.asarray(ref_acc, np.float64)
    tol = rel * np.abs(ref_acc) + amb + ACC_ABS
    n, m = ref_acc.shape
    exact = 0
    exempt = 0
    col = np.broadcast_to(np.arange(m), (n, m))
    order = np.lexsort((col, -ref_acc), axis=1)[:, :k]
    for r in range(n):
        gi = [int(j) for j in gpu_idx[r] if j >= 0]
        assert all(j < m for j in gi), (r, gi)
        assert len(set(gi)) == len(gi), (r, gi)
        assert (gpu_idx[r, len(gi):] == -1).all() and (gpu_val[r, len(gi):] == 0).all(), r
        ro = [int(j) for j in order[r] if ref_acc[r, j] > 0]
        if gi == ro:
            exact += 1
        else:
            exempt += 1
            sg, so = set(gi), set(ro)
            # every entry the GPU chose must be positive within tolerance
            for j in gi:
                assert ref_acc[r, j] + tol[r, j] > 0, (r, j)
            # swapped-in and swapped-out entries must be near-tied
            for j in sg - so:
                for jj in so - sg:
                    assert abs(ref_acc[r, j] - ref_acc[r, jj]) <= tol[r, j] + tol[r, jj], \
                        (r, j, jj, ref_acc[r, j], ref_acc[r, jj])
            # the GPU may keep fewer/more only where the missing ones are ~0
            if len(gi) < len(ro):
                for jj in so - sg:
                    assert ref_acc[r, jj] <= tol[r, jj] or \
                        any(abs(ref_acc[r, jj] - ref_acc[r, j]) <= tol[r, jj] + tol[r, j] for j in gi), (r, jj)
        # order: a later GPU entry may not exceed an earlier one beyond tolerance
        for a in range(len(gi)):
            for b in range(a + 1, len(gi)):
                ja, jb = gi[a], gi[b]
                assert ref_acc[r, ja] >= ref_acc[r, jb] - tol[r, ja] - tol[r, jb], (r, gi)
        # values, normalised over the GPU's own set
        if gi:
            s = ref_acc[r, gi].sum()
            want = ref_acc[r, gi] / s
            vt = rel * want + (amb[r, gi] + want * amb[r, gi].sum()) / s + 1e-7
            got = np.asarray(gpu_val[r, :len(gi)], np.float64)
            assert (np.abs(got - want) <= vt).all(), (r, got, want)
    return dict(rows=n, exact=exact, exempt=exempt)
