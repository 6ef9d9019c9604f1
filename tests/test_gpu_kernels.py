"""GPU parity of the kernels behind the C-ABI against the oracle (MI355X).

K1 (stencil block matvec) against oracle.operator.apply_operator; K4 (dense
eigen-decomposition) against LAPACK's eigenvalues and the eigen-equation.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _fields(nx, ny, nz, seed, h=0.5):
    from oracle import operator as op
    rng = np.random.default_rng(seed)
    V = rng.uniform(-4.0, 1.0, nx * ny * nz)
    ab = (0.5, 2.0, 0.0, 0.4, 1.7, (nz - 1) * h)
    gL, gR = op.gamma_fields(nx, ny, nz, h, ab)
    return V, ab, gL, gR


def _to_dev(torch, X, pad):
    """(N, B) host block -> (B, N) device view whose rows sit `pad` elements apart beyond N."""
    N, B = X.shape
    buf = torch.zeros((B, N + pad), dtype={np.complex128: torch.complex128,
                                            np.complex64: torch.complex64}[X.dtype.type], device="cuda")
    buf[:, :N] = torch.tensor(np.ascontiguousarray(X.T), device="cuda")
    return buf[:, :N]


# shapes cover a tile of the x extent (16, 32 and 64 wide), ragged tiles in
# x and y, z shorter than the finite-difference reach, and padded columns
@pytest.mark.parametrize("shape,B,R,pad", [((10, 10, 20), 16, 6, 0), ((13, 11, 17), 5, 6, 3), ((7, 9, 30), 3, 6, 0),
                                           ((12, 12, 12), 8, 3, 0), ((5, 6, 7), 1, 1, 0), ((32, 32, 64), 16, 6, 64),
                                           ((70, 19, 9), 2, 6, 0), ((64, 40, 33), 3, 6, 0), ((33, 17, 5), 2, 4, 1)])
def test_stencil_c128_matches_oracle(torch_cuda, shape, B, R, pad):
    torch = torch_cuda
    from oracle import operator as op
    from paper_1606_01139_amd import Operator
    nx, ny, nz = shape
    print(f"stencil c128 shape={shape} B={B} R={R} pad={pad}", flush=True)
    V, ab, gL, gR = _fields(nx, ny, nz, 3)
    N = nx * ny * nz
    rng = np.random.default_rng(4)
    X = rng.standard_normal((N, B)) + 1j * rng.standard_normal((N, B))
    ref = op.apply_operator(nx, ny, nz, 0.5, V, gL, gR, X, R)
    oper = Operator(nx, ny, nz, 0.5, V, ab, fd_radius=R)
    Xd = _to_dev(torch, X, pad)
    Yd = _to_dev(torch, np.zeros_like(X), pad)
    oper.apply(Xd, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy().T
    scale = np.abs(ref).max()
    assert np.abs(Y - ref).max() <= 1e-13 * scale


@pytest.mark.parametrize("shape,B", [((10, 10, 20), 16), ((13, 11, 17), 5), ((32, 32, 64), 16), ((64, 64, 40), 2)])
def test_stencil_c64_matches_oracle(torch_cuda, shape, B):
    torch = torch_cuda
    from oracle import operator as op
    from paper_1606_01139_amd import Operator
    nx, ny, nz = shape
    print(f"stencil c64 shape={shape} B={B}", flush=True)
    V, ab, gL, gR = _fields(nx, ny, nz, 5)
    N = nx * ny * nz
    rng = np.random.default_rng(6)
    X = (rng.standard_normal((N, B)) + 1j * rng.standard_normal((N, B))).astype(np.complex64)
    ref = op.apply_operator(nx, ny, nz, 0.5, V, gL, gR, X.astype(np.complex128), 6)
    oper = Operator(nx, ny, nz, 0.5, V, ab)
    Xd = _to_dev(torch, X, 0)
    Yd = _to_dev(torch, np.zeros_like(X), 0)
    oper.apply(Xd, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy().T.astype(np.complex128)
    # FP32 accumulation over 37 taps: relative error a few ulp of float32
    assert np.abs(Y - ref).max() <= 1e-6 * np.abs(ref).max()


# every geometry the autotuner may pick: tile widths 16/32/64, one or two
# points per thread in y, z chunks shorter and longer than the grid, launch
# order and XCD-grouped order, on ragged tiles in x and y (block counts that
# are not multiples of 8, so the padded XCD grid has idle workgroups)
@pytest.mark.parametrize("tx,yb,zc,xcd,nt", [(16, 1, 16, 0, 512), (16, 2, 24, 1, 512), (32, 2, 5, 0, 512),
                                             (32, 2, 5, 1, 512), (64, 2, 48, 0, 512), (32, 1, 192, 1, 512),
                                             (64, 1, 7, 0, 512), (64, 1, 7, 1, 512), (16, 1, 16, 1, 256),
                                             (16, 2, 9, 0, 256), (32, 1, 5, 1, 256), (32, 2, 48, 1, 256)])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_stencil_tuned_geometries_match_oracle(torch_cuda, tmp_path, tx, yb, zc, xcd, nt, dtype):
    torch = torch_cuda
    from oracle import operator as op
    from paper_1606_01139_amd import Operator
    from paper_1606_01139_amd.binding import load_tuning
    nx, ny, nz, B = 37, 29, 21, 3
    print(f"stencil geometry tx={tx} yb={yb} zchunk={zc} xcd={xcd} nt={nt} {dtype}", flush=True)
    elem = 16 if dtype == "c128" else 8
    f = tmp_path / "tune.json"
    f.write_text('{"stencil": [{"nx": %d, "ny": %d, "nz": %d, "cols": %d, "elem": %d, "radius": 6, "tx": %d, '
                 '"yb": %d, "zchunk": %d, "xcd": %d, "nt": %d, "us": 0}]}' % (nx, ny, nz, B, elem, tx, yb, zc, xcd, nt))
    assert load_tuning(str(f)) == 1
    from paper_1606_01139_amd.binding import stencil_geometry, C128, C64
    used = stencil_geometry(nx, ny, nz, B, C128 if dtype == "c128" else C64)
    assert used == {"tx": tx, "yb": yb, "zchunk": min(zc, nz), "xcd": xcd, "nt": nt, "cb": 1, "tuned": True}, used
    V, ab, gL, gR = _fields(nx, ny, nz, 8)
    N = nx * ny * nz
    rng = np.random.default_rng(9)
    X = rng.standard_normal((N, B)) + 1j * rng.standard_normal((N, B))
    if dtype == "c64":
        X = X.astype(np.complex64)
    ref = op.apply_operator(nx, ny, nz, 0.5, V, gL, gR, X.astype(np.complex128), 6)
    oper = Operator(nx, ny, nz, 0.5, V, ab)
    Xd = _to_dev(torch, X, 0)
    Yd = _to_dev(torch, np.zeros_like(X), 0)
    oper.apply(Xd, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy().T.astype(np.complex128)
    tol = 1e-13 if dtype == "c128" else 1e-6
    assert np.abs(Y - ref).max() <= tol * np.abs(ref).max()
    oper.close()


# two columns per thread (complex64): odd and even column counts (the last
# group of an odd count has one column), both block sizes and orders
@pytest.mark.parametrize("tx,yb,zc,xcd,nt,B", [(32, 1, 16, 0, 512, 3), (64, 2, 7, 1, 512, 4), (16, 2, 24, 1, 256, 5),
                                              (32, 2, 48, 0, 256, 1)])
def test_stencil_two_columns_per_thread_match_oracle(torch_cuda, tmp_path, tx, yb, zc, xcd, nt, B):
    torch = torch_cuda
    from oracle import operator as op
    from paper_1606_01139_amd import Operator
    from paper_1606_01139_amd.binding import load_tuning, stencil_geometry, C64
    nx, ny, nz = 37, 29, 21
    print(f"stencil two columns per thread tx={tx} yb={yb} zchunk={zc} xcd={xcd} nt={nt} B={B}", flush=True)
    f = tmp_path / "tune.json"
    f.write_text('{"stencil": [{"nx": %d, "ny": %d, "nz": %d, "cols": %d, "elem": 8, "radius": 6, "tx": %d, '
                 '"yb": %d, "zchunk": %d, "xcd": %d, "nt": %d, "cb": 2, "us": 0}]}' % (nx, ny, nz, B, tx, yb, zc, xcd, nt))
    assert load_tuning(str(f)) == 1
    used = stencil_geometry(nx, ny, nz, B, C64)
    assert used == {"tx": tx, "yb": yb, "zchunk": min(zc, nz), "xcd": xcd, "nt": nt, "cb": 2, "tuned": True}, used
    V, ab, gL, gR = _fields(nx, ny, nz, 8)
    N = nx * ny * nz
    rng = np.random.default_rng(19)
    X = (rng.standard_normal((N, B)) + 1j * rng.standard_normal((N, B))).astype(np.complex64)
    ref = op.apply_operator(nx, ny, nz, 0.5, V, gL, gR, X.astype(np.complex128), 6)
    oper = Operator(nx, ny, nz, 0.5, V, ab)
    Xd = _to_dev(torch, X, 0)
    Yd = _to_dev(torch, np.zeros_like(X), 0)
    oper.apply(Xd, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy().T.astype(np.complex128)
    assert np.abs(Y - ref).max() <= 1e-6 * np.abs(ref).max()
    oper.close()


def test_stencil_autotuner_picks_a_candidate_and_keeps_parity(torch_cuda, tmp_path):
    torch = torch_cuda
    from oracle import operator as op
    from paper_1606_01139_amd import Operator
    from paper_1606_01139_amd.binding import load_tuning
    nx, ny, nz, B = 20, 24, 40, 4
    print("stencil autotuner", flush=True)
    V, ab, gL, gR = _fields(nx, ny, nz, 11)
    oper = Operator(nx, ny, nz, 0.5, V, ab)
    out = tmp_path / "tuned.json"
    geo, us = oper.tune_stencil(B, 0, 3, str(out))
    assert geo["tx"] in (16, 32, 64) and geo["yb"] in (1, 2) and 1 <= geo["zchunk"] <= nz and geo["tried"] > 10
    assert us > 0
    assert load_tuning(str(out)) >= 1
    from paper_1606_01139_amd.binding import stencil_geometry
    used = stencil_geometry(nx, ny, nz, B, 0)
    assert used["tuned"] and all(used[k] == geo[k] for k in ("tx", "yb", "zchunk", "xcd", "nt", "cb")), (used, geo)
    N = nx * ny * nz
    X = np.random.default_rng(12).standard_normal((N, B)) + 0.5j
    ref = op.apply_operator(nx, ny, nz, 0.5, V, gL, gR, X, 6)
    Xd = _to_dev(torch, X, 0)
    Yd = _to_dev(torch, np.zeros_like(X), 0)
    oper.apply(Xd, Yd)
    torch.cuda.synchronize()
    assert np.abs(Yd.cpu().numpy().T - ref).max() <= 1e-13 * np.abs(ref).max()
    oper.close()


@pytest.mark.parametrize("m,batch", [(1, 1), (2, 2), (8, 3), (37, 2), (128, 2), (304, 1), (600, 1)])
def test_dense_eig_matches_lapack(torch_cuda, m, batch):
    torch = torch_cuda
    from paper_1606_01139_amd import dense_eig
    print(f"dense_eig m={m} batch={batch}", flush=True)
    rng = np.random.default_rng(m)
    # Rayleigh-Ritz-like: Hermitian part plus a small negative-imaginary PSD part
    Hs = []
    for _ in range(batch):
        X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        Hh = (X + X.conj().T) / 2
        G = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        Hs.append(Hh - 0.05j * (G @ G.conj().T) / m)
    H = np.stack(Hs)
    Hd = torch.tensor(H, device="cuda")
    th, Y, info = dense_eig(Hd)
    torch.cuda.synchronize()
    th, Y, info = th.cpu().numpy(), Y.cpu().numpy(), info.cpu().numpy()
    assert (info == 0).all()
    for b in range(batch):
        ref = np.linalg.eigvals(H[b])
        nrm = np.linalg.norm(H[b], 2)
        # each computed eigenvalue matches a distinct LAPACK eigenvalue
        d = np.abs(th[b][:, None] - ref[None, :])
        from scipy.optimize import linear_sum_assignment
        r, c = linear_sum_assignment(d)
        assert d[r, c].max() <= 1e-11 * max(nrm, 1.0)
        # eigen-equation residual and unit norm
        R = H[b] @ Y[b] - Y[b] * th[b][None, :]
        assert np.abs(R).max() <= 1e-11 * max(nrm, 1.0)
        np.testing.assert_allclose(np.linalg.norm(Y[b], axis=0), 1.0, atol=1e-12)


def test_dense_eig_rejects_basis_above_maximum(torch_cuda):
    # A Hessenberg row must fit one wavefront's registers (14 values per
    # lane, m <= 896); a larger m is refused on the host before any launch.
    torch = torch_cuda
    from paper_1606_01139_amd import TsgError, dense_eig
    from paper_1606_01139_amd.binding import STATUS_NAMES
    print("dense_eig m=897 (rejected on the host)", flush=True)
    H = torch.zeros((1, 897, 897), dtype=torch.complex128, device="cuda")
    with pytest.raises(TsgError) as err:
        dense_eig(H)
    assert STATUS_NAMES[err.value.status] == "TSG_EINVAL"
    assert "896" in str(err.value)


def test_dense_eig_chase_helpers_match_single_workgroup_chase(torch_cuda, monkeypatch):
    # From m = 128 on, each window's Schur chase runs with helper workgroups
    # that replay the rotations above and to the right of the bulge train;
    # TSG_SCHUR_HELPERS=0 keeps the whole chase in one workgroup.  Both apply
    # the same rotations to every element in the same order, so the spectra
    # agree to rounding, and both must be eigenpairs of H.  8 x 450 is the
    # shape of the c2 solve (50 pairs per window, 8 windows).
    torch = torch_cuda
    from scipy.optimize import linear_sum_assignment
    from paper_1606_01139_amd import dense_eig
    rng = np.random.default_rng(450)
    m, batch = 450, 8
    Hs = []
    for _ in range(batch):
        X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        Hs.append((X + X.conj().T) / 2 - 0.05j * (X @ X.conj().T) / m)
    H = np.stack(Hs)
    print("dense_eig 8 x 450, chase with helpers", flush=True)
    monkeypatch.delenv("TSG_SCHUR_HELPERS", raising=False)
    th0, Y0, info0 = dense_eig(torch.tensor(H, device="cuda"))
    torch.cuda.synchronize()
    print("dense_eig 8 x 450, one workgroup per chase", flush=True)
    monkeypatch.setenv("TSG_SCHUR_HELPERS", "0")
    th1, Y1, info1 = dense_eig(torch.tensor(H, device="cuda"))
    torch.cuda.synchronize()
    monkeypatch.delenv("TSG_SCHUR_HELPERS")
    assert (info0.cpu().numpy() == 0).all() and (info1.cpu().numpy() == 0).all()
    th0, th1, Y0 = th0.cpu().numpy(), th1.cpu().numpy(), Y0.cpu().numpy()
    for b in range(batch):
        nrm = np.linalg.norm(H[b], 2)
        d = np.abs(th0[b][:, None] - th1[b][None, :])
        r, c = linear_sum_assignment(d)
        assert d[r, c].max() <= 1e-12 * nrm
        R = H[b] @ Y0[b] - Y0[b] * th0[b][None, :]
        assert np.abs(R).max() <= 1e-11 * nrm


def test_dense_eig_log_flush_path_is_identical(torch_cuda, monkeypatch):
    # The Schur chase logs its rotations and a second kernel applies them to
    # the Schur vectors; when the log is full the chase applies it itself.
    # With a 5-step log that path runs many times per matrix and must give
    # the same eigenvalues and vectors, bit for bit (same operations, same
    # order per element).
    torch = torch_cuda
    from paper_1606_01139_amd import dense_eig
    rng = np.random.default_rng(5)
    m, batch = 100, 2
    Hs = []
    for _ in range(batch):
        X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        Hs.append((X + X.conj().T) / 2 - 0.05j * (X @ X.conj().T) / m)
    H = np.stack(Hs)
    print("dense_eig with a 5-step rotation log", flush=True)
    monkeypatch.delenv("TSG_SCHUR_LOG_STEPS", raising=False)
    th0, Y0, info0 = dense_eig(torch.tensor(H, device="cuda"))
    torch.cuda.synchronize()
    monkeypatch.setenv("TSG_SCHUR_LOG_STEPS", "5")
    th1, Y1, info1 = dense_eig(torch.tensor(H, device="cuda"))
    torch.cuda.synchronize()
    monkeypatch.delenv("TSG_SCHUR_LOG_STEPS")
    assert (info0.cpu().numpy() == 0).all() and (info1.cpu().numpy() == 0).all()
    assert np.array_equal(th0.cpu().numpy(), th1.cpu().numpy())
    assert np.array_equal(Y0.cpu().numpy(), Y1.cpu().numpy())
    for b in range(batch):
        R = H[b] @ Y1[b].cpu().numpy() - Y1[b].cpu().numpy() * th1[b].cpu().numpy()[None, :]
        assert np.abs(R).max() <= 1e-11 * max(np.linalg.norm(H[b], 2), 1.0)
