"""Test-only NumPy interpreter of a lowered program (qc_plan_describe JSON).

It runs the program's steps on the CPU exactly as the device executes them --
each GEMM step reads its operands' flat storage as [nb][m][k] (or [nb][k][m])
and [nb][k][n] (or [nb][n][k]) and writes [nb][m][n], scattered into its
output tensor's layout when that differs (c_nat != c) -- so a planner or
lowering mistake (a wrong index class, layout, transpose or stride flag)
shows up on the CPU, separately from kernel bugs.  It also evaluates each
step a second way, by einsum over index ids, as a check of the first.

With ``flat=True`` every tensor lives in one buffer at the offset the
program gives it, poisoned with NaN beforehand, and the operations run in the
device's order (leaves, then the micro steps, which read their operands as
produced, then the other steps), so a liveness or aliasing mistake -- a
tensor overwritten while still needed, or read before it is written --
changes the result or leaves a NaN in it.

It is not a fallback of the library: the library never calls it.
"""

import numpy as np


def _open_segments(desc):
    oq = set(desc.get("open_qubits", []))
    return {e for e, s in enumerate(desc["segments"]) if s[2] >= 0 and s[2] in oq}


def _leaf_tensor(desc, leaf, bitstrings, chunk_base):
    segs = desc["segments"]
    bs_base = desc["bs_base"]
    b = desc["b"]
    m = desc["m"]
    sliced = desc["sliced"]
    open_segs = _open_segments(desc)
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
            if segs[e][2] >= 0 and e not in open_segs:
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


def _einsum_step(get, layouts, a, b, c):
    la, lb, lc = layouts[a], layouts[b], layouts[c]
    ids = {}
    for e in la + lb + lc:
        ids.setdefault(e, len(ids))
    ea = get(a).reshape([2] * len(la)) if la else get(a).reshape(())
    eb = get(b).reshape([2] * len(lb)) if lb else get(b).reshape(())
    return ea, eb, np.einsum(ea, [ids[e] for e in la], eb, [ids[e] for e in lb], [ids[e] for e in lc])


def run_program(desc, bitstrings, chunk_base=0, check_einsum=True, flat=False):
    """Root values of one chunk: complex128 [2^b, 2^m], or [2^b, 2^m, 2^n_open]
    for a plan with open output qubits."""
    layouts = [t["layout"] for t in desc["tensors"]]
    if flat:
        arena = np.full(max(1, desc["tensor_elems"]), np.nan + 1j * np.nan, dtype=np.complex128)

        def get(t):
            off = desc["tensors"][t]["offset"]
            return arena[off:off + (1 << len(layouts[t]))].copy()

        def put(t, v):
            off = desc["tensors"][t]["offset"]
            arena[off:off + (1 << len(layouts[t]))] = v
    else:
        tensors = {}

        def get(t):
            return tensors[t]

        def put(t, v):
            tensors[t] = v

    for leaf in desc["leaves"]:
        put(leaf["tensor"], _leaf_tensor(desc, leaf, bitstrings, chunk_base))
    ops = desc["ops"]
    if flat:
        ops = [op for op in ops if op["micro"]] + [op for op in ops if not op["micro"]]
    for op in ops:
        if op["op"] == "transpose":
            if flat and op["micro"]:
                continue  # its consumer is a micro step, which reads the source as produced
            src, dst = op["src"], op["dst"]
            ls, ld = layouts[src], layouts[dst]
            a = get(src).reshape([2] * len(ls)) if ls else get(src)
            put(dst, np.ascontiguousarray(np.transpose(a, [ls.index(e) for e in ld])).reshape(-1))
            continue
        if flat and op["micro"]:
            # The micro-step kernel contracts by index strides of the operands as produced.
            _, _, ref = _einsum_step(get, layouts, op["a_src"], op["b_src"], op["c"])
            put(op["c"], np.ascontiguousarray(ref).reshape(-1))
            continue
        nb, m, n, k = op["nb"], op["m"], op["n"], op["k"]
        A = get(op["a"]).reshape(nb, k, m).transpose(0, 2, 1) if op["a_km"] else get(op["a"]).reshape(nb, m, k)
        B = get(op["b"]).reshape(nb, n, k).transpose(0, 2, 1) if op["b_nk"] else get(op["b"]).reshape(nb, k, n)
        C = np.matmul(A, B).reshape(-1)
        nat = op.get("c_nat", op["c"])
        if nat != op["c"]:
            # The step writes its natural [batch][m][n] order scattered
            # into the layout of tensor c.
            ln, lc = layouts[nat], layouts[op["c"]]
            C = np.ascontiguousarray(np.transpose(C.reshape([2] * len(ln)), [ln.index(e) for e in lc])).reshape(-1)
        if check_einsum:
            ea, eb, ref = _einsum_step(get, layouts, op["a"], op["b"], op["c"])
            # Rounding of a k-term sum is bounded by k |A|max |B|max.
            scale = k * np.abs(ea).max(initial=0.0) * np.abs(eb).max(initial=0.0)
            assert np.abs(ref.reshape(-1) - C).max(initial=0.0) <= 1e-13 * scale, \
                "GEMM view disagrees with einsum"
        put(op["c"], C)
    root = get(desc["root"])
    n_open = len(desc.get("open_qubits", []))
    if n_open:
        return root.reshape(1 << desc["b"], 1 << desc["m"], 1 << n_open)
    return root.reshape(1 << desc["b"], 1 << desc["m"])


def sliced_amplitudes(desc, bitstrings, n_slices, flat=False):
    """Sum over all slices (chunks of 2^b) of the root values: [n_bs] complex
    (or [n_bs, 2^n_open] with open outputs), and the per-slice values."""
    chunk = 1 << desc["b"]
    n_open = len(desc.get("open_qubits", []))
    shape = (len(bitstrings),) + ((1 << n_open,) if n_open else ())
    total = np.zeros(shape, dtype=np.complex128)
    per_slice = np.zeros((n_slices,) + shape, dtype=np.complex128)
    for cb in range(0, n_slices, chunk):
        r = run_program(desc, bitstrings, cb, flat=flat)
        per_slice[cb:cb + chunk] = r[:, :len(bitstrings)]
        total += r[:, :len(bitstrings)].sum(axis=0)
    return total, per_slice


def check_liveness(desc):
    """Static check of the program's buffer offsets in the device's order
    (leaves, micro steps, other steps): every tensor written while another
    one is still to be read (including by the same step) must not overlap
    it.  Returns the number of writes checked."""
    T = desc["tensors"]
    ops = [op for op in desc["ops"] if op["micro"]] + [op for op in desc["ops"] if not op["micro"]]
    ops = [op for op in ops if not (op["op"] == "transpose" and op["micro"])]
    reads, writes = [], []
    for op in ops:
        if op["op"] == "transpose":
            reads.append([op["src"]])
            writes.append(op["dst"])
        elif op["micro"]:
            reads.append([op["a_src"], op["b_src"]])
            writes.append(op["c"])
        else:
            reads.append([op["a"], op["b"]])
            writes.append(op["c"])
    n = len(ops)
    last_read = {}
    for i, rs in enumerate(reads):
        for t in rs:
            last_read[t] = i
    last_read[desc["root"]] = n  # read by the copy after the last step
    born = {leaf["tensor"]: -1 for leaf in desc["leaves"]}

    def span(t):
        off = T[t]["offset"]
        return off, off + (1 << len(T[t]["layout"]))

    checked = 0
    for i, w in enumerate(writes):
        lo, hi = span(w)
        for t, b in born.items():
            if t == w or last_read.get(t, -2) < i:
                continue  # dead (or never read) by the time step i writes
            tlo, thi = span(t)
            assert hi <= tlo or thi <= lo, f"step {i} writes tensor {w} over live tensor {t}"
        for t in reads[i]:
            assert t in born, f"step {i} reads tensor {t} before it is written"
        born[w] = i
        checked += 1
    assert desc["root"] in born
    return checked
