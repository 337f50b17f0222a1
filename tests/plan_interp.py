"""Test-only NumPy interpreter of a lowered program (qc_plan_describe JSON).

It runs the program's steps on the CPU exactly as the device executes them --
each GEMM step reads its operands' flat storage as [nb][m][k] (or [nb][k][m])
and [nb][k][n] (or [nb][n][k]) and writes [nb][m][n], scattered into its
output tensor's layout when that differs (c_nat != c) -- so a planner or
lowering mistake (a wrong index class, layout, transpose or stride flag)
shows up on the CPU, separately from kernel bugs.  It also evaluates each
step a second way, by einsum over index ids, as a check of the first.  It is
not a fallback of the library: the library never calls it.
"""

import numpy as np


def _leaf_tensor(desc, leaf, bitstrings, chunk_base):
    segs = desc["segments"]
    bs_base = desc["bs_base"]
    b = desc["b"]
    m = desc["m"]
    sliced = desc["sliced"]
    fixed = {e: j for j, e in enumerate(sliced) if j >= b}
    idx = leaf["idx"]
    base = (np.asarray(leaf["re"]) + 1j * np.asarray(leaf["im"])).reshape([2] * len(idx)) if idx else \
        np.asarray(leaf["re"][0] + 1j * leaf["im"][0])
    layout = desc["tensors"][leaf["tensor"]]["layout"]
    n_bs_pad = 1 << m
    has_bs = any(e >= bs_base for e in layout)
    kept = [e for e in layout if e < bs_base]
    blocks = []
    for bs in range(n_bs_pad if has_bs else 1):
        sel = []
        for e in idx:
            if segs[e][2] >= 0:
                q = segs[e][2]
                x = bitstrings[bs] if bs < len(bitstrings) else np.zeros_like(bitstrings[0])
                sel.append(int(x[q]))
            elif e in fixed:
                sel.append((int(chunk_base) >> fixed[e]) & 1)
            else:
                sel.append(slice(None))
        sub = base[tuple(sel)] if idx else base
        rest = [e for e in idx if not isinstance(sel[idx.index(e)], int)]
        perm = [rest.index(e) for e in kept]
        blocks.append(np.transpose(sub, perm) if perm else np.asarray(sub))
    if has_bs:
        arr = np.stack(blocks, axis=0).reshape([2] * m + [2] * len(kept))
        # bitstring bits are the leading indices kBsBase + m - 1 ... kBsBase + 0
        cur = [bs_base + i for i in range(m - 1, -1, -1)] + kept
        perm = [cur.index(e) for e in layout]
        arr = np.transpose(arr, perm)
    else:
        arr = blocks[0]
    return np.ascontiguousarray(arr, dtype=np.complex128).reshape(-1)


def run_program(desc, bitstrings, chunk_base=0, check_einsum=True):
    """Returns root values as complex128 [2^b, 2^m] for one chunk."""
    tensors = {}
    layouts = [t["layout"] for t in desc["tensors"]]
    for leaf in desc["leaves"]:
        tensors[leaf["tensor"]] = _leaf_tensor(desc, leaf, bitstrings, chunk_base)
    for op in desc["ops"]:
        if op["op"] == "transpose":
            src, dst = op["src"], op["dst"]
            ls, ld = layouts[src], layouts[dst]
            a = tensors[src].reshape([2] * len(ls)) if ls else tensors[src]
            tensors[dst] = np.ascontiguousarray(np.transpose(a, [ls.index(e) for e in ld])).reshape(-1)
        else:
            nb, m, n, k = op["nb"], op["m"], op["n"], op["k"]
            A = tensors[op["a"]].reshape(nb, k, m).transpose(0, 2, 1) if op["a_km"] else \
                tensors[op["a"]].reshape(nb, m, k)
            B = tensors[op["b"]].reshape(nb, n, k).transpose(0, 2, 1) if op["b_nk"] else \
                tensors[op["b"]].reshape(nb, k, n)
            C = np.matmul(A, B).reshape(-1)
            nat = op.get("c_nat", op["c"])
            if nat != op["c"]:
                # The step writes its natural [batch][m][n] order scattered
                # into the layout of tensor c.
                ln, lc = layouts[nat], layouts[op["c"]]
                C = np.ascontiguousarray(np.transpose(C.reshape([2] * len(ln)), [ln.index(e) for e in lc])).reshape(-1)
            if check_einsum:
                la, lb, lc = layouts[op["a"]], layouts[op["b"]], layouts[op["c"]]
                ids = {}
                for e in la + lb + lc:
                    ids.setdefault(e, len(ids))
                ea = tensors[op["a"]].reshape([2] * len(la)) if la else tensors[op["a"]].reshape(())
                eb = tensors[op["b"]].reshape([2] * len(lb)) if lb else tensors[op["b"]].reshape(())
                ref = np.einsum(ea, [ids[e] for e in la], eb, [ids[e] for e in lb], [ids[e] for e in lc])
                # Rounding of a k-term sum is bounded by k |A|max |B|max.
                scale = k * np.abs(ea).max(initial=0.0) * np.abs(eb).max(initial=0.0)
                assert np.abs(ref.reshape(-1) - C).max(initial=0.0) <= 1e-13 * scale, \
                    "GEMM view disagrees with einsum"
            tensors[op["c"]] = C
    root = tensors[desc["root"]]
    return root.reshape(1 << desc["b"], 1 << desc["m"])


def sliced_amplitudes(desc, bitstrings, n_slices):
    """Sum over all slices (chunks of 2^b) of the root values: [n_bs] complex."""
    chunk = 1 << desc["b"]
    total = np.zeros(len(bitstrings), dtype=np.complex128)
    per_slice = np.zeros((n_slices, len(bitstrings)), dtype=np.complex128)
    for cb in range(0, n_slices, chunk):
        r = run_program(desc, bitstrings, cb)
        per_slice[cb:cb + chunk] = r[:, :len(bitstrings)]
        total += r[:, :len(bitstrings)].sum(axis=0)
    return total, per_slice
