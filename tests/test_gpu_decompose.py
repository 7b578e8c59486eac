"""GPU parity: FWHT Pauli decomposition and pruning vs the oracle.

Bar: coefficients within 1e-13 absolute; the kept index set and its order
bit-exact (ranking ties broken by flat index); relative Frobenius error
within 1e-12.
"""
import numpy as np
import pytest

from oracle import pauli as op
from workloads import heleshaw_like, random_symmetric, toeplitz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2604_14435_amd import api  # noqa: E402
from paper_2604_14435_amd import _lib as L  # noqa: E402

DEV = "cuda:0"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _flat(strings, n):
    s = strings.cpu().numpy().astype(np.int64)
    return s[:, 0] * (1 << n) + s[:, 1]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 8, 9, 10, 11])
def test_dense_matches_oracle_random(n):
    """Every coefficient; n <= 9 runs the tiled two-pass transform, n = 10, 11
    the single fused pass."""
    A = random_symmetric(n, seed=n)
    A[0, -1] += 0.3  # break the symmetry: odd-Y strings become nonzero
    got = api.pauli_decompose_dense(_gpu(A)).cpu().numpy()
    want = op.decompose_fwht(A)
    assert np.max(np.abs(got - want)) < 1e-13


def test_dense_toeplitz_n10_closed_form_values():
    n = 10
    A = toeplitz(n, 1.0, -0.45)
    got = api.pauli_decompose_dense(_gpu(A)).cpu().numpy()
    want = op.decompose_fwht(A)
    assert np.max(np.abs(got - want)) < 1e-13
    assert np.count_nonzero(np.abs(got) > 1e-15) == 1 << n


def test_dense_n12_random_symmetric_sampled_rows():
    """The 4096 x 4096 dense symmetric N(0,1) matrix: 24 sampled x-rows
    recomputed one by one with the oracle's transform."""
    n = 12
    N = 1 << n
    A = random_symmetric(n, seed=0)
    got = api.pauli_decompose_dense(_gpu(A))
    rng = np.random.default_rng(7)
    xs = np.concatenate([[0, 1, N - 1], rng.integers(0, N, 21)])
    k = np.arange(N)
    for x in xs:
        w = op.walsh_hadamard(A[k ^ x, k])
        ny = np.bitwise_count(np.uint64(x) & k.astype(np.uint64)).astype(np.int64) % 4
        want = np.array([1, -1j, -1, 1j])[ny] * w / N
        row = got[int(x)].cpu().numpy()
        assert np.max(np.abs(row - want)) < 1e-13, x
    # Parseval over the whole output
    tot = float((got.abs() ** 2).sum().item()) * N
    assert abs(tot - np.sum(A * A)) < 1e-9 * np.sum(A * A)


@pytest.mark.parametrize("b,tau,L_expect", [(-0.45, 0.01, 64), (-0.45, 0.005, 128), (-1 / 3, 0.1, 4),
                                             (-1 / 3, 0.005, 128)])
def test_tau_selection_toeplitz_n10(b, tau, L_expect):
    n = 10
    A = toeplitz(n, 1.0, b)
    coeffs, strings, ferr = api.pauli_decompose(_gpu(A), tau=tau)
    C = op.decompose_fwht(A)
    keep = op.select_tau(C, tau)
    assert len(keep) == L_expect == coeffs.shape[0]
    assert np.array_equal(_flat(strings, n), keep)
    assert np.max(np.abs(coeffs.cpu().numpy() - C.ravel()[keep])) < 1e-13
    assert abs(ferr - op.frobenius_error(C, keep, A)) < 1e-12


@pytest.mark.parametrize("L_", [1, 63, 64, 100, 1024, 1500])
def test_top_L_with_ties_toeplitz(L_):
    """Cuts inside a group of equal magnitudes: the index tie-break decides."""
    n = 10
    A = toeplitz(n, 1.0, -1 / 3)
    coeffs, strings, ferr = api.pauli_decompose(_gpu(A), top_L=L_)
    C = op.decompose_fwht(A)
    keep = op.select_top(C, L_)
    assert np.array_equal(_flat(strings, n), keep)
    assert np.max(np.abs(coeffs.cpu().numpy() - C.ravel()[keep])) < 1e-13
    assert abs(ferr - op.frobenius_error(C, keep, A)) < 1e-12


def test_top_L_heleshaw_like():
    """The Hele-Shaw-like pressure operator (32 x 32 grid), top 256."""
    A, _ = heleshaw_like(32, 0.5, seed=0)
    n = 10
    coeffs, strings, ferr = api.pauli_decompose(_gpu(A), top_L=256)
    C = op.decompose_fwht(A)
    keep = op.select_top(C, 256)
    mag = np.sort(np.abs(C.ravel()))[::-1]
    assert mag[255] - mag[256] > 1e-12  # the cut is not a near-tie
    assert np.array_equal(_flat(strings, n), keep)
    assert np.max(np.abs(coeffs.cpu().numpy() - C.ravel()[keep])) < 1e-13
    assert abs(ferr - op.frobenius_error(C, keep, A)) < 1e-12


def test_top_L_random_n8_and_edge_cases():
    n = 8
    A = random_symmetric(n, seed=11)
    C = op.decompose_fwht(A)
    c, s, f = api.pauli_decompose(_gpu(A), top_L=4 ** n + 5)  # more than exist: all
    assert c.shape[0] == 4 ** n
    assert np.array_equal(_flat(s, n), op.select_top(C, 4 ** n))
    assert f == 0.0
    c, s, f = api.pauli_decompose(_gpu(A), tau=1e6)  # nothing kept
    assert c.shape[0] == 0 and abs(f - 1.0) < 1e-12
    c, s, f = api.pauli_decompose(_gpu(A), top_L=300)
    assert np.array_equal(_flat(s, n), op.select_top(C, 300))


def test_capacity_error_reports_count():
    n = 10
    A = toeplitz(n, 1.0, -0.45)
    with pytest.raises(L.DvqError) as e:
        api.pauli_decompose(_gpu(A), tau=0.01, capacity=10)
    assert e.value.status == L.DVQ_ECAPACITY
    assert "64 kept" in str(e.value)


def test_n1_smallest():
    A = np.array([[2.0, -0.5], [0.25, 1.0]])
    got = api.pauli_decompose_dense(_gpu(A)).cpu().numpy()
    assert np.max(np.abs(got - op.decompose_bruteforce(A))) < 1e-15


@pytest.mark.parametrize("n,L_", [(3, 8), (6, 20), (10, 64)])
def test_pauli_sum_dense_reconstructs(n, L_):
    """sum_l c_l P_l against the oracle's Kronecker-product reconstruction;
    with every term kept (n = 3) it returns A itself."""
    A = random_symmetric(n, seed=n) if n < 10 else toeplitz(n, 1.0, -0.45)
    C = op.decompose_fwht(A)
    keep = op.select_top(C, L_ if n > 3 else 4 ** n)
    c, xs, zs = op.kept_terms(C, keep)
    strings = np.stack([xs, zs], 1).astype(np.int32)
    got = api.pauli_sum_dense(_gpu(c), _gpu(strings), n).cpu().numpy()
    want = op.reconstruct(c, xs, zs, n)
    assert np.max(np.abs(got - want)) < 1e-13
    if n == 3:
        assert np.max(np.abs(got - A)) < 1e-13


def test_batch_matches_single_calls():
    """The batched top-L decomposition of a family equals one call per matrix
    (n = 8, seven systems, L = 40: a cut inside some Toeplitz levels, where
    the index tie-break decides) and the oracle."""
    n, L_ = 8, 40
    mats = [toeplitz(n, 1.0 + 0.05 * i, -0.45 + 0.04 * i) for i in range(7)]
    mats[3] = random_symmetric(n, seed=3)
    c, s, f = api.pauli_decompose_batch(_gpu(np.stack(mats)), L_)
    for i, A in enumerate(mats):
        c1, s1, f1 = api.pauli_decompose(_gpu(A), top_L=L_)
        assert torch.equal(c[i], c1) and torch.equal(s[i], s1) and f[i] == f1
        C = op.decompose_fwht(A)
        keep = op.select_top(C, L_)
        assert np.array_equal(_flat(s[i], n), keep)
        assert abs(f[i] - op.frobenius_error(C, keep, A)) < 1e-12


def test_device_toeplitz_batches_equal_host_recipe():
    """The warm-start family built in device memory equals
    workloads.toeplitz element by element, and decomposes to the same terms."""
    from paper_2604_14435_amd.warmstart import decompose_batches, decompose_family, toeplitz_batches
    from workloads import toeplitz_family

    n = 7
    ab = toeplitz_family(11, seed=3)
    dev_mats = torch.cat(list(toeplitz_batches(ab, n, DEV, chunk=4)))
    host = np.stack([toeplitz(n, a, b) for a, b in ab])
    assert np.array_equal(dev_mats.cpu().numpy(), host)
    c1, s1, f1 = decompose_batches(toeplitz_batches(ab, n, DEV, chunk=4), 24)
    c2, s2, f2 = decompose_family((toeplitz(n, a, b) for a, b in ab), 24, DEV, chunk=5)
    assert torch.equal(c1, c2) and torch.equal(s1, s2) and np.array_equal(f1, f2)
