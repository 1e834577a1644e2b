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


def ht_from_dev(H, T, d):
    """Read back an HT written by slar_truncate into numpy (oracle layout)."""
    rk = list(H.rank)
    L = [T["leaves"][m][: T["leaves"][m].shape[0]].cpu().numpy().ravel()[: T["leaves"][m].shape[0] * rk[m]]
         .reshape(T["leaves"][m].shape[0], rk[m]) for m in range(d)]
    out = {"leaves": L}
    if d == 2:
        out["root"] = T["root"].cpu().numpy().ravel()[: rk[0] * rk[1]].reshape(rk[0], rk[1])
    else:
        r1, r2, r3, r4, r12, r34 = rk
        out["B12"] = T["B12"].cpu().numpy().ravel()[: r1 * r2 * r12].reshape(r1, r2, r12)
        out["B34"] = T["B34"].cpu().numpy().ravel()[: r3 * r4 * r34].reshape(r3, r4, r34)
        out["root"] = T["root"].cpu().numpy().ravel()[: r12 * r34].reshape(r12, r34)
    return out
