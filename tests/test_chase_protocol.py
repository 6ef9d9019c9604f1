"""The split of one multishift sweep between the chase workgroup and its
helpers (smallqr.hip), modelled on the CPU.

A sweep chases bulges j = 0..ns-1, bulge j at row p = lo + s - 3 j at step
s, each step a left rotation on rows p, p+1 (columns from p-1, or lo, to
the right) and a right rotation on columns p, p+1 (rows up to p+2).  In a
deferred sweep the chase keeps rows from rlo(s) = max(lo, lo + s - 3(ns-1))
down and columns up to e(s) = min(ihi, lo + 32 (s // 32 + 2)); a helper owns
32 rows and the 32 columns of the same indices and replays the logged
rotations onto them in passes of up to 32 published steps: a row from
srow(r) on, a column before scol(c) (never given back beyond ihi).  Records
are published every 8 steps; the chase takes 32 columns back every 32 steps
once their helpers have replayed every earlier step.

The model replays that schedule with helpers run at random points allowed
by what has been published, and checks that
  * H after the sweep equals the plain sweep's bit for bit (each element
    takes the same rotations in the same order);
  * every rotation a helper applies falls inside the segment its pass
    staged;
  * no helper pass holds an element (from the step at which it can start,
    until the chase next waits for it) that the chase reads or writes, and
    no two helpers hold the same element at once.
Columns beyond ihi take all left rotations (the column replay's share in a
sweep without helpers).

A second model follows one column of H beyond every ihi and one row of Z
through a whole run of blocks, deferred steps taking effect when the
helpers replay them and the rest when the replays run (or the chase
flushes its log), and checks that the result is that of log order."""
import random

import numpy as np
import pytest

TAKE, BAND, CHUNK, PUB = 32, 32, 32, 8


def givens(x, y):
    nx2, ny2 = abs(x) ** 2, abs(y) ** 2
    if ny2 == 0:
        return 1.0, 0j
    if nx2 == 0:
        return 0.0, np.conj(y) / np.sqrt(ny2)
    ir, ix = 1 / np.sqrt(nx2 + ny2), 1 / np.sqrt(nx2)
    return nx2 * ix * ir, (ix * ir) * (x * np.conj(y))


def left(c, s, a, b):
    return c * a + s * b, c * b - np.conj(s) * a


def right(c, s, a, b):
    return c * a + np.conj(s) * b, c * b - s * a


def sweep(H, lo, ihi, shifts, deferred, rng=None):
    m = H.shape[0]
    H = H.copy()
    ns = len(shifts)
    nsteps = (ihi - lo) + 3 * (ns - 1)
    nh = (m + BAND - 1) // BAND
    srow = lambda r: 0 if r < lo else r - lo + 3 * (ns - 1) + 1
    scol = lambda c: 0 if c < lo else ((1 << 30) if c > ihi else TAKE * max(0, (c - lo + TAKE - 1) // TAKE - 2))
    log, done, passes = [], [0] * nh, []
    touched = {}  # element -> steps at which the chase reads or writes it

    def touch(e, s):
        touched.setdefault(e, []).append(s)

    def helper(h, upto):
        while done[h] < upto:
            sa = done[h]
            sb = min(upto, sa + CHUNK)
            base, top = max(lo, lo + sa - 3 * (ns - 1)), min(ihi, lo + sb)
            held = {}
            for x in range(h * BAND, min(m, (h + 1) * BAND)):
                if srow(x) < sb:
                    seg = H[x, base:top + 1].copy()
                    for q in range(top - base + 1):
                        held[(x, base + q)] = nsteps
                    for s in range(max(sa, srow(x)), sb):
                        for (c, p, sj) in log[s]:
                            if p >= 0:
                                assert base <= p and p + 1 <= top
                                seg[p - base], seg[p + 1 - base] = right(c, sj, seg[p - base], seg[p + 1 - base])
                    H[x, base:top + 1] = seg
                if scol(x) > sa:
                    seg = H[base:top + 1, x].copy()
                    for q in range(top - base + 1):
                        held[(base + q, x)] = scol(x)
                    for s in range(sa, min(sb, scol(x))):
                        for (c, p, sj) in log[s]:
                            if p >= 0:
                                assert base <= p and p + 1 <= top
                                seg[p - base], seg[p + 1 - base] = left(c, sj, seg[p - base], seg[p + 1 - base])
                    H[base:top + 1, x] = seg
            passes.append((h, sb - 1, held))
            done[h] = sb

    published = 0
    for step in range(nsteps):
        recs = []
        for j in range(ns):
            p = lo + step - 3 * j
            if lo <= p < ihi:
                if p == lo:
                    x, y = H[lo, lo] - shifts[j], H[lo + 1, lo]
                    touch((lo, lo), step)
                    touch((lo + 1, lo), step)
                else:
                    x, y = H[p, p - 1], H[p + 1, p - 1]
                    touch((p, p - 1), step)
                    touch((p + 1, p - 1), step)
                c, sj = givens(x, y)
                recs.append((c, p, sj))
            else:
                recs.append((1.0, -1, 0j))
        log.append(recs)
        ecol, rlo = ihi, 0
        if deferred:
            if (step + 1) % PUB == 0 or step + 1 == nsteps:
                published = step + 1
            for h in range(nh):
                if rng.random() < 0.3:
                    helper(h, rng.randint(done[h], max(done[h], published)))
            ecol = min(ihi, lo + TAKE * (step // TAKE + 2))
            rlo = max(lo, lo + step - 3 * (ns - 1))
            first = lo + TAKE * (step // TAKE + 1) + 1
            if step > 0 and step % TAKE == 0 and first <= ecol:
                assert published >= step  # the step before a take was published
                for h in range(first // BAND, ecol // BAND + 1):
                    helper(h, published)
        else:
            # columns beyond ihi: what the column replay applies afterwards
            for (c, p, sj) in recs:
                if p >= 0:
                    for col in range(ihi + 1, m):
                        H[p, col], H[p + 1, col] = left(c, sj, H[p, col], H[p + 1, col])
        for (c, p, sj) in recs:  # all left rotations of the step
            if p < 0:
                continue
            for col in range(p - 1 if p > lo else lo, ecol + 1):
                a, b = left(c, sj, H[p, col], H[p + 1, col])
                H[p, col], H[p + 1, col] = a, (0 if col == p - 1 else b)
                touch((p, col), step)
                touch((p + 1, col), step)
        for (c, p, sj) in recs:  # then all right rotations
            if p < 0:
                continue
            for r in range(rlo, min(p + 2, ihi) + 1):
                H[r, p], H[r, p + 1] = right(c, sj, H[r, p], H[r, p + 1])
                touch((r, p), step)
                touch((r, p + 1), step)
    if deferred:
        for h in range(nh):
            helper(h, nsteps)
        holders = {}
        for (h, start, held) in passes:
            for e, until in held.items():
                for s in touched.get(e, []):
                    assert not (start <= s < until), (h, start, e, s, until)
                holders.setdefault(e, []).append((h, start, until))
        for e, lst in holders.items():
            for i in range(len(lst)):
                for k in range(i + 1, len(lst)):
                    (h1, a1, b1), (h2, a2, b2) = lst[i], lst[k]
                    assert h1 == h2 or b1 <= a2 or b2 <= a1, (e, lst[i], lst[k])
    return H


@pytest.mark.parametrize("m,lo,ihi,ns", [(160, 0, 130, 16), (200, 5, 199, 9), (300, 37, 250, 16)])
def test_deferred_sweep_matches_plain_sweep(m, lo, ihi, ns):
    r = np.random.default_rng(m + lo)
    H = np.triu(r.standard_normal((m, m)) + 1j * r.standard_normal((m, m)), -1)
    shifts = r.standard_normal(ns) + 1j * r.standard_normal(ns)
    plain = sweep(H, lo, ihi, shifts, False)
    for seed in (1, 2):
        split = sweep(H, lo, ihi, shifts, True, random.Random(seed))
        assert np.array_equal(plain, split)


def _order_model(m, blocks, flush_rule, rng):
    """One column of H beyond every ihi and one row of Z under a whole
    Schur run: blocks of (lo, ihi, sweeps, deferred, finished), each sweep
    a list of steps of disjoint rotations on the block, a finished block
    ended by a unitary on its rows (the LDS finish; a block that splits has
    none, its parts follow).  Steps of deferred sweeps take effect when
    the helpers replay them; the rest when the replays run after the kernel,
    or when the chase flushes its log (before a deferred sweep, if the log
    holds steps of an undeferred sweep of a block of 128 or more rows).
    Returns (in log order, as the protocol applies them)."""
    col_ref = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    zrow_ref = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    col, zrow = col_ref.copy(), zrow_ref.copy()
    pending, nd_log = [], False

    def apply(op, col, zrow):
        kind, a, b = op
        if kind == "rot":  # left rotation on rows (a, a+1); right rotation on Z columns (a, a+1)
            c, s = b
            col[a], col[a + 1] = left(c, s, col[a], col[a + 1])
            zrow[a], zrow[a + 1] = right(c, s, zrow[a], zrow[a + 1])
        else:  # unitary Q on rows / Z columns [a, a + n)
            Q = b
            n = Q.shape[0]
            col[a:a + n] = Q.conj().T @ col[a:a + n]
            zrow[a:a + n] = zrow[a:a + n] @ Q

    def flush():
        nonlocal pending, nd_log
        for op in pending:
            apply(op, col, zrow)
        pending, nd_log = [], False

    for (lo, ihi, nsweeps, deferred, finished) in blocks:
        for _ in range(nsweeps):
            if deferred and flush_rule and nd_log:
                flush()
            for s in range(8):
                ps = range(lo + (s % 3), ihi, 3)
                for p in ps:
                    c, sj = givens(rng.standard_normal() + 1j * rng.standard_normal(),
                                   rng.standard_normal() + 1j * rng.standard_normal())
                    op = ("rot", p, (c, sj))
                    apply(op, col_ref, zrow_ref)
                    if deferred:
                        apply(op, col, zrow)
                    else:
                        pending.append(op)
            if not deferred and ihi - lo + 1 >= 128:
                nd_log = True
        if not finished:
            continue
        X = rng.standard_normal((ihi - lo + 1,) * 2) + 1j * rng.standard_normal((ihi - lo + 1,) * 2)
        Q, _ = np.linalg.qr(X)
        op = ("q", lo, Q)
        apply(op, col_ref, zrow_ref)
        pending.append(op)
    flush()
    return col_ref, zrow_ref, col, zrow


def test_replays_keep_log_order():
    # blocks in the order the chase meets them: [0, 299] swept first without
    # helpers (they had not started), then with them, until it splits at 250
    # and 200; [250, 299] and [200, 249], too small for helpers, are swept
    # and finished; then [0, 199] with helpers
    m = 300
    blocks = [(0, 299, 1, False, False), (0, 299, 2, True, False), (250, 299, 2, False, True),
              (200, 249, 1, False, True), (0, 199, 2, True, True)]
    ref_c, ref_z, col, zrow = _order_model(m, blocks, True, np.random.default_rng(3))
    np.testing.assert_allclose(col, ref_c, rtol=0, atol=1e-12)
    np.testing.assert_allclose(zrow, ref_z, rtol=0, atol=1e-12)
    # without the flush the undeferred sweep of [0, 299] would be replayed
    # after the deferred ones that overlap it
    ref_c, ref_z, col, zrow = _order_model(m, blocks, False, np.random.default_rng(3))
    assert np.abs(col - ref_c).max() > 1e-6
