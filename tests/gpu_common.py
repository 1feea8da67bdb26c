"""Helpers shared by the GPU parity tests (no test functions here)."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2308_13476_amd import _binding as B
    B.lib()  # fail loudly when the HIP library is missing


def dev():
    return torch.device("cuda:0")


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def to_np(t):
    return t.detach().cpu().numpy()


def stencil_to_csr(st: np.ndarray) -> sp.csr_matrix:
    """[(2r+1)^2, m, m] stencil planes (coefficient of node (i,j) -> (i+dx, j+dy)) to a sparse matrix."""
    D = int(round(np.sqrt(st.shape[0])))
    r = D // 2
    m = st.shape[1]
    rows, cols, vals = [], [], []
    J, I = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    for d in range(D * D):
        dx, dy = d % D - r, d // D - r
        K, L = I + dx, J + dy
        ok = (K >= 0) & (K < m) & (L >= 0) & (L < m) & (st[d] != 0)
        rows.append((J * m + I)[ok])
        cols.append((L * m + K)[ok])
        vals.append(st[d][ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m * m, m * m))


def rel(a, b):
    """Normwise relative difference ||a - b||_2 / ||b||_2."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def node_rel(a, b):
    """Largest difference at any single node relative to the largest value,
    max_p |a_p - b_p| / max_p |b_p|: a wrong boundary row or corner, which the
    2-norm over a million nodes could hide, shows here at full size."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def level_shape(n_l):
    return (n_l + 1, n_l + 1)
