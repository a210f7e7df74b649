"""Run as a child process by test_gpu_torch.py: torch is imported before libkth.so
(the order the two HIP runtimes need in one process), then the autograd function
of the binding is checked against the oracle gradient and central differences."""
import os
import sys

import numpy as np
import torch  # noqa: F401  (first)

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_1710_05134_amd as K  # noqa: E402
import pencilgen as pg  # noqa: E402
from oracle import dense as od  # noqa: E402


def main():
    ctx = K.Context(0)
    p = pg.tb_supercell((2, 2, 2), seed=11)
    k = p.n // 2
    print(f"autograd kth_eig n={p.n} k={k}", flush=True)
    P = K.Pencil.from_pencilgen(ctx, p)
    opts = K.default_opts(start_vectors=pg.start_vectors(p.n))
    F = K.eig_function()
    a = torch.tensor(p.a_val, dtype=torch.float64, requires_grad=True)
    b = torch.tensor(p.b_val, dtype=torch.float64, requires_grad=True)
    lam = F.apply(a, b, P, k, opts)
    (3.0 * lam).backward()
    lam_ref, x_ref = od.kth(p, k)
    ga_ref, gb_ref = od.hf_gradient(p, lam_ref, x_ref)
    nA = od.norm_inf(p)
    assert abs(lam.item() - lam_ref) <= 1e-10 * nA
    assert np.max(np.abs(a.grad.numpy() - 3.0 * ga_ref)) <= 3e-8 * np.max(np.abs(ga_ref))
    assert np.max(np.abs(b.grad.numpy() - 3.0 * gb_ref)) <= 3e-8 * np.max(np.abs(gb_ref))
    # central differences of the forward on symmetric pairs of stored entries of A
    # (each stored entry is its own variable: the pair's derivative is g_q + g_q')
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    xr = x_ref[rows] * x_ref[p.col]
    cand = np.nonzero((rows < p.col) & (np.abs(xr) > 1e-3 * np.abs(xr).max()))[0]
    h = 1e-6
    for q in np.random.default_rng(3).choice(cand, 4, replace=False):
        i, j = rows[q], p.col[q]
        q2 = p.rowptr[j] + int(np.searchsorted(p.col[p.rowptr[j]:p.rowptr[j + 1]], i))
        vals = []
        for sgn in (1, -1):
            av = p.a_val.copy()
            av[q] += sgn * h
            av[q2] += sgn * h
            vals.append(F.apply(torch.tensor(av), torch.tensor(p.b_val), P, k, opts).item())
        fd = (vals[0] - vals[1]) / (2 * h)
        an = (a.grad[q].item() + a.grad[q2].item()) / 3.0
        assert abs(fd - an) <= 1e-7 + 1e-4 * abs(an), (i, j, fd, an)
        print(f"  pair ({i},{j}): fd {fd:.9f} autograd {an:.9f}", flush=True)
    # device tensors: the same lambda_k bit for bit, the same gradients, on the GPU
    a_d = torch.tensor(p.a_val, dtype=torch.float64, device="cuda", requires_grad=True)
    b_d = torch.tensor(p.b_val, dtype=torch.float64, device="cuda", requires_grad=True)
    lam_d = F.apply(a_d, b_d, P, k, opts)
    (3.0 * lam_d).backward()
    assert lam_d.is_cuda and lam_d.item() == lam.item()
    assert a_d.grad.is_cuda
    assert np.array_equal(a_d.grad.cpu().numpy(), a.grad.numpy())
    assert np.array_equal(b_d.grad.cpu().numpy(), b.grad.numpy())
    print("  device tensors: same lambda_k and gradients", flush=True)
    # the library's device memory from torch's caching allocator
    before = torch.cuda.memory_allocated(0)
    ctx_t = K.Context(0, torch_allocator=True)
    P_t = K.Pencil.from_pencilgen(ctx_t, p)
    lam_t, _, info_t = P_t.eig(k, opts=opts)
    held = torch.cuda.memory_allocated(0) - before
    assert info_t["k_validated"] == k and lam_t == lam.item(), (lam_t, lam.item())
    assert held > 0, held
    P_t.close()
    ctx_t.close()
    print(f"  torch caching allocator: same lambda_k, {held} bytes held through torch", flush=True)
    print("autograd check ok", flush=True)


if __name__ == "__main__":
    main()
