"""tsg_dense_eig_noalloc (the fixed-scratch variant of tsg_dense_eig for
callers that cannot allocate) against tsg_dense_eig: the same kernels on
the same inputs, so the outputs must be identical, on two calls in a row
(the second smaller, so it runs over what the first left in the scratch);
and a batch beyond the scratch is refused before anything is launched."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _matrices(batch, m, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(batch):
        X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        # Rayleigh-Ritz-like: Hermitian part plus a small negative-imaginary part
        out.append((X + X.conj().T) / 2 - 0.05j * (X @ X.conj().T) / m)
    return np.stack(out)


def test_noalloc_dense_eig_matches_allocating_call(torch_cuda):
    torch = torch_cuda
    from paper_1606_01139_amd.binding import dense_eig, dense_eig_noalloc
    for batch, m, seed in [(3, 300, 1), (2, 96, 2)]:
        print(f"noalloc dense_eig batch={batch} m={m}", flush=True)
        H0 = torch.tensor(_matrices(batch, m, seed), device="cuda")
        th_ref, Y_ref, info_ref = dense_eig(H0.clone())
        H = H0.clone()
        th = torch.empty((batch, m), dtype=torch.complex128, device="cuda")
        Y = torch.empty((batch, m, m), dtype=torch.complex128, device="cuda")
        info = torch.full((batch,), -7, dtype=torch.int32, device="cuda")
        dense_eig_noalloc(H, th, Y, info)
        torch.cuda.synchronize()
        assert torch.equal(info, info_ref) and int(info.abs().sum()) == 0
        assert torch.equal(th, th_ref)
        assert torch.equal(Y, Y_ref)
        # and they are eigenpairs: ||H y - theta y|| small for unit y
        Hn = H0.cpu().numpy()
        Yn, tn = Y.cpu().numpy(), th.cpu().numpy()
        for b in range(batch):
            r = Hn[b] @ Yn[b] - Yn[b] * tn[b][None, :]
            assert np.abs(r).max() <= 1e-10 * np.abs(Hn[b]).max() * m


def test_noalloc_dense_eig_refuses_batches_beyond_the_scratch(torch_cuda):
    torch = torch_cuda
    from paper_1606_01139_amd.binding import dense_eig_noalloc, TsgError, TSG_EINVAL
    batch, m = 3, 450  # 3 x 27.5 MB of workspace > 64 MiB
    H = torch.zeros((batch, m, m), dtype=torch.complex128, device="cuda")
    th = torch.zeros((batch, m), dtype=torch.complex128, device="cuda")
    Y = torch.zeros((batch, m, m), dtype=torch.complex128, device="cuda")
    info = torch.full((batch,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(TsgError) as e:
        dense_eig_noalloc(H, th, Y, info)
    assert e.value.status == TSG_EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert int(info[0]) == -7  # nothing was launched
