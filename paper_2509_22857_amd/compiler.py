"""Post-training model compiler: turns a trained polynomial CNN (batch
normalisations, activations with any leading coefficient, average pooling)
into the network description the encrypted evaluator runs.

Passes, in the order the paper applies them (Sections 4 and 5):
  fuse          node fusing, Section 4.1 Cases 1-4 (closed forms derived in the
                appendix on node fusing);
  redistribute  weight redistribution, Section 4.2: every polynomial becomes
                monic and every pooling divisor becomes 1, with compensating
                updates forward (to consumers) or backward (to producers),
                per the appendix on weight redistribution;
  lower         slice / slice-ensemble clustering of every convolution
                (Section 5.2-5.3) and emission of the evaluator's network
                description (the dict `GpuNetwork` consumes).

Graph form (host side, float64; every parameter carries a leading axis over
the M ensemble members, M = 1 for a single network):

  graph = {"members": M, "image": (C, H, W), "nodes": [node, ...]}

nodes in topological order, each {"op", "name", "inp": [tensor, ...],
"out": tensor, **params}; the input tensor is "x", the graph's output is the
last node's "out".  Operations:

  conv     W [M][O][I][k][k], b [M][O] or None, stride: zero-padded 'same'
           convolution (output H // stride; output row r reads input rows
           stride r + dh - k // 2)
  dense    W [M][K][C], b [M][K] or None, on a channel vector
  scale    s [M][C]: diagonal kernel y_c = s_c x_c (an explicit identity
           shortcut)
  bn       gamma, beta, mean, var [M][C], eps: B(x) = b1 x + b0 with
           b1 = gamma / sqrt(var + eps), b0 = beta - b1 mean
  poly     c [M][C][d + 1]: sum_i c_i x^i per channel
  bipoly   c [M][C][3][3]: sum_{i + j <= 2} c_ij x^i y^j, inputs (x, y)
  add      two inputs of equal shape
  avgpool  div: 2x2 window, stride 2, sum / div (div 4 is the average)
  gap      div: sum over the grid / div (div H W is global average pooling)

poly, bipoly, avgpool and gap may carry "absorb" [M][C]: their output is
multiplied by it.  Redistribution leaves it only on a donor whose output is
the graph's output (nothing downstream can take the update); the evaluator
folds a uniform one into the activation's scale.
"""
from __future__ import annotations

import copy

import numpy as np

KERNELS = ("conv", "dense", "scale")


class CompileError(ValueError):
    pass


# ----------------------------------------------------------------- graph helpers
def producers(nodes):
    return {n["out"]: i for i, n in enumerate(nodes)}


def consumers(nodes):
    cons = {}
    for i, n in enumerate(nodes):
        for t in n["inp"]:
            cons.setdefault(t, []).append(i)
    return cons


def shapes(graph):
    """Tensor name -> shape ((C, H, W) on the grid, (C,) after gap/dense)."""
    sh = {"x": tuple(graph["image"])}
    names = [n["name"] for n in graph["nodes"]]
    outs = [n["out"] for n in graph["nodes"]]
    if len(set(names)) != len(names) or len(set(outs)) != len(outs) or "x" in outs:
        raise CompileError("node names and output tensors must be unique (and not 'x')")
    for n in graph["nodes"]:
        for t in n["inp"]:
            if t not in sh:
                raise CompileError(f"{n['name']}: input {t} is not produced before it")
        s = sh[n["inp"][0]]
        op = n["op"]
        if op == "conv":
            O, I, k = n["W"].shape[1], n["W"].shape[2], n["W"].shape[3]
            if I != s[0] or k % 2 == 0:
                raise CompileError(f"{n['name']}: weights {n['W'].shape[1:]} do not fit input {s}")
            sh[n["out"]] = (O, s[1] // n["stride"], s[2] // n["stride"])
        elif op == "dense":
            if len(s) != 1 or n["W"].shape[2] != s[0]:
                raise CompileError(f"{n['name']}: dense on a {s} tensor")
            sh[n["out"]] = (n["W"].shape[1],)
        elif op == "avgpool":
            sh[n["out"]] = (s[0], s[1] // 2, s[2] // 2)
        elif op == "gap":
            sh[n["out"]] = (s[0],)
        elif op in ("add", "bipoly"):
            if sh[n["inp"][1]] != s:
                raise CompileError(f"{n['name']}: inputs {s} and {sh[n['inp'][1]]} differ")
            sh[n["out"]] = s
        else:
            sh[n["out"]] = s
    return sh


def _bn_affine(n):
    b1 = n["gamma"] / np.sqrt(n["var"] + n["eps"])
    return b1, n["beta"] - b1 * n["mean"]


def _sole_consumer(nodes, t, i):
    """True when node i is the only reader of tensor t."""
    return consumers(nodes).get(t, []) == [i]


# ----------------------------------------------------------------- node fusing (Section 4.1)
def fuse_case1(b1, b0, c):
    """Case 1, P(B(x)) -> P(x): c = (c0, c1, c2) per channel on the last axis."""
    c0, c1, c2 = c[..., 0], c[..., 1], c[..., 2]
    return np.stack([b0 * b0 * c2 + b0 * c1 + c0, b1 * (2.0 * b0 * c2 + c1), b1 * b1 * c2], axis=-1)


def fuse_case2(b1, b0, W, beta):
    """Case 2, B(C(x)) -> C(x): weights scaled per output channel by b1, bias
    b1 beta + b0.  W [M][O][...], beta [M][O] or None."""
    Wf = W * b1.reshape(b1.shape + (1,) * (W.ndim - 2))
    return Wf, b1 * (0.0 if beta is None else beta) + b0


def fuse_case3(bx1, bx0, by1, by0, c):
    """Case 3, P(B_X(x) + B_Y(y)) -> S(x, y); returns c_ij [..][3][3]."""
    c0, c1, c2 = c[..., 0], c[..., 1], c[..., 2]
    s0 = bx0 + by0
    S = np.zeros(c.shape[:-1] + (3, 3))
    S[..., 2, 0] = c2 * bx1 * bx1
    S[..., 0, 2] = c2 * by1 * by1
    S[..., 1, 1] = 2.0 * c2 * bx1 * by1
    S[..., 1, 0] = bx1 * (2.0 * c2 * s0 + c1)
    S[..., 0, 1] = by1 * (2.0 * c2 * s0 + c1)
    S[..., 0, 0] = c2 * s0 * s0 + c1 * s0 + c0
    return S


def fuse_case4(bx1, bx0, c):
    """Case 4, P(B_X(x) + y) -> S(x, y) (identity shortcut)."""
    c0, c1, c2 = c[..., 0], c[..., 1], c[..., 2]
    S = np.zeros(c.shape[:-1] + (3, 3))
    S[..., 2, 0] = c2 * bx1 * bx1
    S[..., 0, 2] = c2
    S[..., 1, 1] = 2.0 * c2 * bx1
    S[..., 1, 0] = bx1 * (2.0 * c2 * bx0 + c1)
    S[..., 0, 1] = 2.0 * c2 * bx0 + c1
    S[..., 0, 0] = c2 * bx0 * bx0 + c1 * bx0 + c0
    return S


def _fold_bn_into_kernels(g, log):
    """Case 2 wherever a batch normalisation reads a convolution (or dense
    layer) that nothing else reads."""
    nodes = g["nodes"]
    changed = True
    while changed:
        changed = False
        prod = producers(nodes)
        for i, n in enumerate(nodes):
            if n["op"] != "bn" or n["inp"][0] not in prod:
                continue
            j = prod[n["inp"][0]]
            k = nodes[j]
            if k["op"] not in ("conv", "dense") or not _sole_consumer(nodes, k["out"], i):
                continue
            b1, b0 = _bn_affine(n)
            k["W"], k["b"] = fuse_case2(b1, b0, k["W"], k.get("b"))
            k["out"] = n["out"]
            del nodes[i]
            log.append(("case2", n["name"], k["name"]))
            changed = True
            break


def _fusable_bn(nodes, t, reader):
    """Index of the batch normalisation producing t if `reader` is its only reader."""
    prod = producers(nodes)
    j = prod.get(t)
    if j is None or nodes[j]["op"] != "bn" or not _sole_consumer(nodes, t, reader):
        return None
    return j


def _fuse_bn_into_polys(g, log):
    """Cases 1, 3 and 4 wherever a quadratic activation reads a batch
    normalisation, or a sum of one or two, that nothing else reads."""
    nodes = g["nodes"]
    changed = True
    while changed:
        changed = False
        prod = producers(nodes)
        for i, n in enumerate(nodes):
            if n["op"] != "poly" or n["c"].shape[-1] != 3:
                continue
            t = n["inp"][0]
            jb = _fusable_bn(nodes, t, i)
            if jb is not None:  # Case 1
                b1, b0 = _bn_affine(nodes[jb])
                n["c"] = fuse_case1(b1, b0, n["c"])
                n["inp"] = [nodes[jb]["inp"][0]]
                log.append(("case1", nodes[jb]["name"], n["name"]))
                del nodes[jb]
                changed = True
                break
            ja = prod.get(t)
            if ja is None or nodes[ja]["op"] != "add" or not _sole_consumer(nodes, t, i):
                continue
            a = nodes[ja]
            jx, jy = (_fusable_bn(nodes, u, ja) for u in a["inp"])
            if jx is None and jy is None:
                continue
            if jx is not None and jy is not None and jx != jy:  # Case 3
                bx1, bx0 = _bn_affine(nodes[jx])
                by1, by0 = _bn_affine(nodes[jy])
                S = fuse_case3(bx1, bx0, by1, by0, n["c"])
                inp = [nodes[jx]["inp"][0], nodes[jy]["inp"][0]]
                gone, case = {ja, jx, jy}, "case3"
            else:  # Case 4: the batch-normalised branch is x, the other y
                if jx is None:
                    jx, y = jy, a["inp"][0]
                else:
                    y = a["inp"][1]
                bx1, bx0 = _bn_affine(nodes[jx])
                S = fuse_case4(bx1, bx0, n["c"])
                inp = [nodes[jx]["inp"][0], y]
                gone, case = {ja, jx}, "case4"
            nodes[i] = dict(op="bipoly", name=n["name"], inp=inp, out=n["out"], c=S)
            log.append((case, a["name"], n["name"]))
            for j in sorted(gone, reverse=True):
                del nodes[j]
            changed = True
            break


def fuse(graph, order: str = "conv_first"):
    """Node fusing.  order "conv_first" folds batch normalisations into the
    preceding convolutions first (Case 2), so a residual sum keeps a
    univariate activation (one ciphertext product); "poly_first" applies
    Cases 1, 3 and 4 first and Case 2 to what is left, as the paper's figure
    groups them.  Returns (graph, log of (case, fused node, into node))."""
    if order not in ("conv_first", "poly_first"):
        raise CompileError(f"unknown fusing order {order!r}")
    g = copy.deepcopy(graph)
    log = []
    passes = (_fold_bn_into_kernels, _fuse_bn_into_polys)
    for p in (passes if order == "conv_first" else passes[::-1]):
        p(g, log)
    return g, log


# ----------------------------------------------------------------- weight redistribution (Section 4.2)
def _explicit_shortcuts(g):
    """Give every input of a sum its own kernel: a sum input not produced by
    a kernel that only the sum reads gets a diagonal scale node (s = 1), so
    that updates reaching a sum land in a kernel (the paper applies them
    consistently along converging branches)."""
    nodes = g["nodes"]
    sh = shapes(g)
    i = 0
    while i < len(nodes):
        n = nodes[i]
        if n["op"] == "add":
            for j, t in enumerate(n["inp"]):
                p = producers(nodes).get(t)
                if p is not None and nodes[p]["op"] in KERNELS and _sole_consumer(nodes, t, i):
                    continue
                s = dict(op="scale", name=f"{n['name']}_in{j}", inp=[t], out=f"{n['name']}_in{j}",
                         s=np.ones((g["members"], sh[t][0])))
                nodes.insert(i, s)
                i += 1
                n["inp"][j] = s["out"]
        i += 1


def _leading(n):
    """The coefficient a donor normalises to 1, or the pooling update."""
    if n["op"] == "poly":
        return n["c"][..., -1]
    if n["op"] == "bipoly":
        return n["c"][..., 2, 0]
    return None


def _is_donor(n):
    if n["op"] == "poly":
        return n["c"].shape[-1] >= 2 and not np.all(n["c"][..., -1] == 1.0)
    if n["op"] == "bipoly":
        return not np.all(n["c"][..., 2, 0] == 1.0)
    return n["op"] in ("avgpool", "gap") and n["div"] != 1


def _receive_forward(g, t, u, log, donor):
    """Consumers of tensor t now read t / u (u [M][C] per channel): update
    them so that every consumer's output is unchanged (forward receivers)."""
    nodes = g["nodes"]
    readers = consumers(nodes).get(t, [])
    if not readers:
        n = nodes[producers(nodes)[t]]
        n["absorb"] = n.get("absorb", 1.0) * u
        log.append(("absorb", donor, n["name"]))
        return
    for i in readers:
        n = nodes[i]
        op = n["op"]
        if op == "conv":
            n["W"] = n["W"] * u[:, None, :, None, None]
        elif op == "dense":
            n["W"] = n["W"] * u[:, None, :]
        elif op == "scale":
            n["s"] = n["s"] * u
        elif op == "bn":  # a degree-1 polynomial: b1 u, b0 unchanged
            n["gamma"], n["mean"] = n["gamma"] * u, n["mean"] / u
        elif op == "poly":
            n["c"] = n["c"] * u[..., None] ** np.arange(n["c"].shape[-1])
        elif op == "bipoly":
            e = np.arange(3)
            if n["inp"][0] == t:
                n["c"] = n["c"] * (u[..., None] ** e)[..., :, None]
            if n["inp"][1] == t:
                n["c"] = n["c"] * (u[..., None] ** e)[..., None, :]
        elif op in ("avgpool", "gap"):  # linear, per channel: the update passes through
            _receive_forward(g, n["out"], u, log, donor)
            continue
        else:
            raise CompileError(f"{n['name']} ({op}) cannot receive an update from {donor}")
        log.append(("forward", donor, n["name"]))


def _pullable(nodes, t, reader):
    """Can tensor t be made u times larger by its producer alone?"""
    p = producers(nodes).get(t)
    if p is None or not _sole_consumer(nodes, t, reader):
        return False
    n = nodes[p]
    if n["op"] in KERNELS or n["op"] == "bn":
        return True
    if n["op"] in ("avgpool", "gap"):
        return _pullable(nodes, n["inp"][0], p)
    if n["op"] == "add":
        return all(_pullable(nodes, s, p) for s in n["inp"])
    return False  # a polynomial producer is a donor already made monic


def _pull(g, t, u, log, donor):
    """Backward receivers: the producer of t now outputs u times as much."""
    nodes = g["nodes"]
    p = producers(nodes)[t]
    n = nodes[p]
    op = n["op"]
    if op == "conv":
        n["W"] = n["W"] * u[:, :, None, None, None]
        n["b"] = None if n.get("b") is None else n["b"] * u
    elif op == "dense":
        n["W"] = n["W"] * u[:, :, None]
        n["b"] = None if n.get("b") is None else n["b"] * u
    elif op == "scale":
        n["s"] = n["s"] * u
    elif op == "bn":
        n["gamma"], n["beta"] = n["gamma"] * u, n["beta"] * u
    elif op in ("avgpool", "gap"):
        _pull(g, n["inp"][0], u, log, donor)
        return
    elif op == "add":
        for s in n["inp"]:
            _pull(g, s, u, log, donor)
        return
    log.append(("backward", donor, n["name"]))


def _normalise(g, i, direction, log):
    n = g["nodes"][i]
    M, C = g["members"], shapes(g)[n["inp"][0]][0]
    op = n["op"]
    if op in ("avgpool", "gap"):
        u = np.full((M, C), 1.0 / n["div"])
        if direction == "backward" and _pullable(g["nodes"], n["inp"][0], i):
            n["div"] = 1
            _pull(g, n["inp"][0], u, log, n["name"])
            log.append(("donor-backward", n["name"], n["name"]))
            return
        n["div"] = 1
        log.append(("donor-forward", n["name"], n["name"]))
        _receive_forward(g, n["out"], u, log, n["name"])
        return
    lead = _leading(n)
    if np.any(lead == 0.0):
        raise CompileError(f"{n['name']}: a zero leading coefficient cannot be normalised")
    d = n["c"].shape[-1] - 1 if op == "poly" else 2
    if direction == "backward" and (d % 2 == 1 or np.all(lead > 0)) and _pullable(g["nodes"], n["inp"][0], i):
        # upsilon = c_d^(1/d); the normalised polynomial reads upsilon x
        u = np.sign(lead) * np.abs(lead) ** (1.0 / d)
        e = np.arange(n["c"].shape[-1] if op == "poly" else 3)
        if op == "poly":
            n["c"] = n["c"] * u[..., None] ** (-e)
            n["c"][..., -1] = 1.0
        else:
            n["c"] = n["c"] * (u[..., None] ** (-e))[..., :, None]
            n["c"][..., 2, 0] = 1.0
        _pull(g, n["inp"][0], u, log, n["name"])
        log.append(("donor-backward", n["name"], n["name"]))
        return
    # forward: upsilon = c_d, the normalised polynomial is P / upsilon
    u = lead.copy()
    if op == "poly":
        n["c"] = n["c"] / u[..., None]
        n["c"][..., -1] = 1.0
    else:
        n["c"] = n["c"] / u[..., None, None]
        n["c"][..., 2, 0] = 1.0
    log.append(("donor-forward", n["name"], n["name"]))
    _receive_forward(g, n["out"], u, log, n["name"])


def redistribute(graph, direction: str = "forward"):
    """Weight redistribution.  Every polynomial (activation, bivariate
    activation) gets leading coefficient 1 and every pooling divisor 1.
    direction "forward" sends each update to the donor's consumers;
    "backward" sends it to the producers where they can take it alone (a
    kernel, or sums and poolings of kernels, that only this path reads; a
    positive leading coefficient when the degree is even) and forward
    otherwise.  Returns (graph, log)."""
    if direction not in ("forward", "backward"):
        raise CompileError(f"unknown direction {direction!r}")
    g = copy.deepcopy(graph)
    _explicit_shortcuts(g)
    log = []
    names = [n["name"] for n in g["nodes"]]
    for name in names:
        i = next(k for k, n in enumerate(g["nodes"]) if n["name"] == name)
        if _is_donor(g["nodes"][i]):
            _normalise(g, i, direction, log)
    return g, log


# ----------------------------------------------------------------- clustering (Section 5.2-5.3)
def lloyd(X: np.ndarray, k: int, seed: int = 0, iters: int = 60):
    """k-means of the rows of X (n x M) under the l2 distance (Lloyd's
    iterations from a k-means++ start).  With n <= k every row is its own
    centroid.  Returns (centroids [k'][M], labels [n])."""
    n = X.shape[0]
    if n <= k:
        return X.copy(), np.arange(n)
    r = np.random.default_rng(seed)
    C = [X[r.integers(n)]]
    d2 = ((X - C[0]) ** 2).sum(axis=1)
    for _ in range(1, k):
        tot = d2.sum()
        j = int(r.integers(n)) if tot == 0.0 else int(np.searchsorted(np.cumsum(d2), r.random() * tot))
        C.append(X[min(j, n - 1)])
        d2 = np.minimum(d2, ((X - C[-1]) ** 2).sum(axis=1))
    C = np.array(C)
    lab = None
    for _ in range(iters):
        d = ((X[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
        new = d.argmin(axis=1)
        if lab is not None and np.array_equal(new, lab):
            break
        lab = new
        for c in range(k):
            sel = lab == c
            if sel.any():
                C[c] = X[sel].mean(axis=0)
    d = ((X[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
    return C, d.argmin(axis=1)


def cluster_slices(W: np.ndarray, k: int, seed: int = 0):
    """Slice-ensemble clustering of W [M][O][I][kh][kw]: for every kernel
    column s the rows of X_s = [(W^(m)_{o,i,h,s})_m] (one per (o, i, h), in
    R^M) share a codebook of at most k centroids.  Returns codebook
    [kw][k][M] (unused entries zero) and indices [O][I][kh][kw] (uint16)."""
    M, O, I, kh, kw = W.shape
    cb = np.zeros((kw, k, M))
    idx = np.zeros((O, I, kh, kw), dtype=np.uint16)
    for s in range(kw):
        X = W[..., s].reshape(M, -1).T
        C, lab = lloyd(X, k, seed=seed * 1009 + s)
        cb[s, :len(C)] = C
        idx[..., s] = lab.reshape(O, I, kh)
    return cb, idx


# ----------------------------------------------------------------- lowering to the evaluator
def _branch(g, t, factor, used):
    """The sum input t as a kernel (W [M][O][I][k][k], bias, stride, input)
    with its output multiplied by factor [M][C]: the producing kernel when
    only this sum reads it (marked used), else a 1x1 diagonal kernel on t."""
    nodes = g["nodes"]
    p = producers(nodes).get(t)
    cons = consumers(nodes).get(t, [])
    if p is not None and len(cons) == 1 and nodes[p]["op"] in ("conv", "scale"):
        n = nodes[p]
        used.add(p)
        if n["op"] == "conv":
            b = None if n.get("b") is None else n["b"] * factor
            return n["W"] * factor[:, :, None, None, None], b, n["stride"], n["inp"][0], n["name"]
        t, base = n["inp"][0], n["s"]
    else:
        base = np.ones_like(factor)
    M, C = factor.shape
    W = np.zeros((M, C, C, 1, 1))
    W[:, np.arange(C), np.arange(C), 0, 0] = base * factor
    return W, None, 1, t, None


def _conv_layer(name, inp, out, W, b, stride, k, seed):
    cb, idx = cluster_slices(W, k, seed)
    return dict(op="conv", name=name, inp=inp, out=out, out_ch=W.shape[1], in_ch=W.shape[2], ksize=W.shape[3],
                stride=stride, codebook=cb, idx=idx, bias=None if b is None else np.array(b, dtype=np.float64))


def _sum_layer(g, name, a, b, fa, fb, out, k, seed, used):
    Wa, ba, sa, ia, na = _branch(g, a, fa, used)
    Wb, bb, sb, ib, nb = _branch(g, b, fb, used)
    if Wb.shape[3] > Wa.shape[3]:  # the wider kernel is the main convolution
        (Wa, ba, sa, ia, na), (Wb, bb, sb, ib, nb) = (Wb, bb, sb, ib, nb), (Wa, ba, sa, ia, na)
    bias = None if ba is None and bb is None else (0.0 if ba is None else ba) + (0.0 if bb is None else bb)
    L = _conv_layer(na or name, ia, out, Wa, bias, sa, k, seed)
    scb, sidx = cluster_slices(Wb, k, seed + 7)
    L["short"] = dict(inp=ib, ksize=Wb.shape[3], stride=sb, out_ch=Wb.shape[1], in_ch=Wb.shape[2], codebook=scb,
                      idx=sidx)
    return L


def _uniform_absorb(n):
    a = np.asarray(n.get("absorb", 1.0), dtype=np.float64)
    if not np.allclose(a, a.flat[0], rtol=1e-12, atol=0.0):
        raise CompileError(f"{n['name']}: the output's scale differs per channel; the evaluator absorbs one "
                           "scale per activation")
    return float(a.flat[0])


def lower(graph, k: int = 64, seed: int = 0, name: str = "compiled", rank_tol: float = 1e-9) -> dict:
    """The evaluator's network description of a fused, redistributed graph.
    Sums of two kernels become a convolution with a shortcut; a bivariate
    activation S(x, y) of Cases 3/4 (monic in x) is lowered as the monic
    univariate activation of z = x + v y, v = c_11 / 2, which requires
    c_02 = v^2 and c_01 = v c_10 -- what Cases 3 and 4 produce."""
    g = copy.deepcopy(graph)
    nodes = g["nodes"]
    sh = shapes(g)
    cons = consumers(nodes)
    M = g["members"]
    layers, used = [], set()
    deferred = set()
    for i, n in enumerate(nodes):  # kernels that a sum or a bivariate activation takes as a branch
        if n["op"] in ("conv", "scale") and len(cons.get(n["out"], [])) == 1:
            r = nodes[cons[n["out"]][0]]
            if r["op"] in ("add", "bipoly"):
                deferred.add(i)
    classes = 0
    for i, n in enumerate(nodes):
        op = n["op"]
        if i in deferred:
            continue
        if op == "bn":
            raise CompileError(f"{n['name']}: batch normalisation left after fusing (not after a convolution, "
                               "nor before an activation)")
        if op == "conv":
            layers.append(_conv_layer(n["name"], n["inp"][0], n["out"], n["W"], n.get("b"), n["stride"], k,
                                      seed + i))
        elif op == "scale":
            C = n["s"].shape[1]
            W = np.zeros((M, C, C, 1, 1))
            W[:, np.arange(C), np.arange(C), 0, 0] = n["s"]
            layers.append(_conv_layer(n["name"], n["inp"][0], n["out"], W, None, 1, k, seed + i))
        elif op == "add":
            one = np.ones((M, sh[n["out"]][0]))
            layers.append(_sum_layer(g, n["name"], n["inp"][0], n["inp"][1], one, one, n["out"], k, seed + i,
                                     used))
        elif op == "poly":
            c = n["c"]
            if c.shape[-1] != 3:
                raise CompileError(f"{n['name']}: degree {c.shape[-1] - 1}; the evaluator runs quadratics")
            if not np.all(c[..., 2] == 1.0):
                raise CompileError(f"{n['name']}: the evaluator runs monic quadratics (redistribute first)")
            layers.append(dict(op="act", name=n["name"], inp=n["inp"][0], out=n["out"], b=c[..., 1].copy(),
                               c=c[..., 0].copy(), a_absorb=_uniform_absorb(n)))
        elif op == "bipoly":
            c = n["c"]
            if not np.all(c[..., 2, 0] == 1.0):
                raise CompileError(f"{n['name']}: bivariate activation not monic in x (redistribute first)")
            v = 0.5 * c[..., 1, 1]
            scale = max(1.0, float(np.abs(c).max()))
            if (np.abs(c[..., 0, 2] - v * v).max() > rank_tol * scale
                    or np.abs(c[..., 0, 1] - v * c[..., 1, 0]).max() > rank_tol * scale):
                raise CompileError(f"{n['name']}: bivariate activation is not a polynomial of x + v y")
            z = f"{n['name']}_z"
            one = np.ones_like(v)
            layers.append(_sum_layer(g, n["name"] + "_sum", n["inp"][0], n["inp"][1], one, v, z, k, seed + i,
                                     used))
            layers.append(dict(op="act", name=n["name"], inp=z, out=n["out"], b=c[..., 1, 0].copy(),
                               c=c[..., 0, 0].copy(), a_absorb=_uniform_absorb(n)))
        elif op == "avgpool":
            if n["div"] != 1:
                raise CompileError(f"{n['name']}: pooling divisor {n['div']} (redistribute first)")
            if _uniform_absorb(n) != 1.0:
                raise CompileError(f"{n['name']}: pooling as the graph's output")
            layers.append(dict(op="pool", name=n["name"], inp=n["inp"][0], out=n["out"]))
        elif op == "gap":
            r = cons.get(n["out"], [])
            if n["div"] != 1 or len(r) != 1 or nodes[r[0]]["op"] != "dense":
                raise CompileError(f"{n['name']}: global pooling must have divisor 1 and feed one dense layer")
        elif op == "dense":
            p = producers(nodes).get(n["inp"][0])
            if p is None or nodes[p]["op"] != "gap":
                raise CompileError(f"{n['name']}: the evaluator's dense layer reads a global sum pooling")
            layers.append(dict(op="dense", name=n["name"], inp=nodes[p]["inp"][0], out=n["out"], w=n["W"].copy(),
                               bias=None if n.get("b") is None else n["b"].copy()))
            classes = n["W"].shape[1]
        else:
            raise CompileError(f"{n['name']}: unknown operation {op}")
    missing = deferred - used
    if missing:
        raise CompileError("kernels left unplaced: " + ", ".join(nodes[i]["name"] for i in sorted(missing)))
    C, H, W = g["image"]
    return dict(name=name, members=M, classes=classes, image=tuple(g["image"]),
                layout=dict(block=1 << int(np.ceil(np.log2(H * W))), row_stride=W), layers=layers, k=k)


def compile_network(graph, k: int = 64, order: str = "conv_first", direction: str = "forward", seed: int = 0,
                    name: str = "compiled"):
    """fuse -> redistribute -> lower.  Returns (network description, log)."""
    shapes(graph)
    g, log1 = fuse(graph, order)
    g, log2 = redistribute(g, direction)
    return lower(g, k=k, seed=seed, name=name), log1 + log2
