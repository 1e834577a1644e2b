"""Helpers shared by the GPU tests: device copies of inputs and the
normwise error of section "error metric" (max|a-b| / max|b|)."""
import numpy as np
import torch


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def ht_to_dev(F, dtype=torch.float64):
    out = {"leaves": [dev(U, dtype) for U in F["leaves"]], "root": dev(F["root"], dtype)}
    if len(F["leaves"]) == 4:
        r1, r2, r12 = F["B12"].shape
        r3, r4, r34 = F["B34"].shape
        out["B12"] = dev(F["B12"].reshape(r1 * r2, r12), dtype)
        out["B34"] = dev(F["B34"].reshape(r3 * r4, r34), dtype)
    return out


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64); b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def ht_from_dev(H, T, d, n):
    """Read back an HT written by slar_truncate (packed leaves [n_m][r_m] at
    the start of each flat buffer) into numpy (oracle layout)."""
    rk = list(H.rank)
    flat = lambda t, cnt: t.reshape(-1)[:cnt].cpu().numpy()   # noqa: E731
    out = {"leaves": [flat(T["leaves"][m], n[m] * rk[m]).reshape(n[m], rk[m]) for m in range(d)]}
    if d == 2:
        out["root"] = flat(T["root"], rk[0] * rk[1]).reshape(rk[0], rk[1])
    else:
        r1, r2, r3, r4, r12, r34 = rk
        out["B12"] = flat(T["B12"], r1 * r2 * r12).reshape(r1, r2, r12)
        out["B34"] = flat(T["B34"], r3 * r4 * r34).reshape(r3, r4, r34)
        out["root"] = flat(T["root"], r12 * r34).reshape(r12, r34)
    return out
