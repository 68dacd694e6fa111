"""Differentiable float32 cumsum (torch.autograd.Function): forward scan and
reverse-scan backward on ragged rows, against the oracle, plus finite
differences.

y = cumsum(x) per row is linear with a lower-triangular all-ones Jacobian, so
dL/dx_i = sum_{j >= i, same row} dL/dy_j (the reverse inclusive scan)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _bound_ok(got, ref, abs_sums):
    return np.all(np.abs(got.astype(np.float64) - ref) <= np.ldexp(abs_sums, -20))


def test_forward_backward_ragged_rows():
    """64 rows, lengths log-uniform in [2^10, 2^22], x and upstream g normal(0,1)."""
    import paper_2312_14874_amd as scan
    x_np, g_np, off = workloads.rows()
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    offs = torch.from_numpy(off).cuda()
    y = scan.cumsum_autograd(x, offs)
    ref_y, ab_y = oracle.segmented_f32(x_np, off)
    assert _bound_ok(y.detach().cpu().numpy(), ref_y, ab_y)
    g = torch.from_numpy(g_np).cuda()
    y.backward(g)
    ref_g, ab_g = oracle.segmented_f32(g_np, off, reverse=True)
    assert _bound_ok(x.grad.cpu().numpy(), ref_g, ab_g)


def test_backward_one_hot_last():
    """A one-hot upstream gradient at a row's last element gives all ones in that row."""
    import paper_2312_14874_amd as scan
    off = np.array([0, 1000, 1000, 5003], dtype=np.int64)
    gy = torch.zeros(5003, device="cuda")
    gy[999] = 1.0
    gy[5002] = 1.0
    gx = scan.cumsum_backward(gy, torch.from_numpy(off).cuda()).cpu().numpy()
    assert np.array_equal(gx, np.ones(5003, dtype=np.float32))


def test_flat_autograd_matches_torch_reference():
    import paper_2312_14874_amd as scan
    n = 300_001
    x_np = workloads.normal_f32(n, seed=3)
    g_np = workloads.normal_f32(n, seed=4)
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    y = scan.cumsum_autograd(x)
    (y * torch.from_numpy(g_np).cuda()).sum().backward()
    ref_g, ab_g = oracle.scan_f32(g_np, reverse=True)
    assert _bound_ok(x.grad.cpu().numpy(), ref_g, ab_g)
    ref_y, ab_y = oracle.scan_f32(x_np)
    assert _bound_ok(y.detach().cpu().numpy(), ref_y, ab_y)


def test_finite_differences_256_rows():
    """Central differences of L(x) = sum_j g_j y_j (accumulated in float64,
    y from the GPU forward) with h = 0.5 against the GPU backward, on 16 rows
    of length 256; one element per row is perturbed per evaluation."""
    import paper_2312_14874_amd as scan
    x2, g2 = workloads.fd_rows()
    rows, L = x2.shape
    off = np.arange(0, rows * L + 1, L, dtype=np.int64)
    offs = torch.from_numpy(off).cuda()
    x = torch.from_numpy(x2.reshape(-1).copy()).cuda()
    g64 = g2.reshape(rows, L).astype(np.float64)

    def loss_rows(xdev):
        y = scan.segmented_scan(xdev, offs).cpu().numpy().astype(np.float64).reshape(rows, L)
        return (y * g64).sum(axis=1)

    gx = scan.cumsum_backward(torch.from_numpy(g2.reshape(-1).copy()).cuda(), offs).cpu().numpy().reshape(rows, L)
    h = np.float32(0.5)
    fd = np.empty((rows, L))
    base = x.clone()
    for i in range(L):
        xp = base.clone()
        xm = base.clone()
        idx = torch.arange(rows, device="cuda") * L + i
        xp[idx] += h
        xm[idx] -= h
        denom = (xp[idx] - xm[idx]).double().cpu().numpy()
        fd[:, i] = (loss_rows(xp) - loss_rows(xm)) / denom
    tol = 1e-3 * (1.0 + np.abs(g64).sum(axis=1, keepdims=True))
    assert np.all(np.abs(fd - gx) <= tol), float(np.abs(fd - gx).max())
    # and the backward against the oracle's suffix sums
    ref, ab = oracle.segmented_f32(g2.reshape(-1), off, reverse=True)
    assert _bound_ok(gx.reshape(-1), ref, ab)


def test_autograd_input_checks():
    import paper_2312_14874_amd as scan
    with pytest.raises(TypeError):
        scan.cumsum_autograd(torch.zeros(10, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        scan.cumsum(torch.zeros(10))   # CPU tensor
