"""Generator of the selection networks used by the HIP kernels.

The kernels compute true (non-separable) window medians -- the paper insists
on the classic median filter rather than a separable approximation (Methods,
"Algorithm"; State of the field) -- on 32-bit integer keys whose signed order is
the float order.  Every median here is a min/max network, so it selects an
input element exactly and is bit-identical to a sort of the window.

Construction, for a k x k window:

* each column of k values is sorted by a small sorting network;
* sorted lists are merged pairwise (Batcher's odd-even merge, or a per-rank
  "merge path" selection, whichever needs fewer live operations) and each
  partial result is trimmed to the ranks that can still be the median: a
  partial set that covers c of the n window values, with t = n - c values
  still to come, can only hold the median at its ranks [med - t, med]
  (every lower rank ends below the median, every higher one above);
* a final backwards liveness pass drops every min or max whose result is not
  needed.

``python gen_median_net.py OUT.h`` writes the header; ``--check`` runs the
self-tests (exhaustive 0-1 inputs for the 3x3 and 5x5 networks, random inputs
with many ties for all of them).
"""

from __future__ import annotations

import itertools
import sys

import numpy as np

# Small sorting networks (comparator lists), each checked by the 0-1 principle.
SORT_NETS = {
    1: [],
    2: [(0, 1)],
    3: [(0, 2), (0, 1), (1, 2)],
    4: [(0, 1), (2, 3), (0, 2), (1, 3), (1, 2)],
    5: [(0, 1), (3, 4), (2, 4), (2, 3), (1, 4), (0, 3), (0, 2), (1, 3), (1, 2)],
    6: [(1, 2), (4, 5), (0, 2), (3, 5), (0, 1), (3, 4), (2, 5), (0, 3), (1, 4), (2, 4),
        (1, 3), (2, 3)],
    7: [(1, 2), (3, 4), (5, 6), (0, 2), (3, 5), (4, 6), (0, 1), (4, 5), (2, 6), (0, 4),
        (1, 5), (0, 3), (2, 5), (1, 3), (2, 4), (2, 3)],
}


class Net:
    """A straight-line network of integer min / max operations."""

    def __init__(self, n_inputs: int):
        self.n_inputs = n_inputs
        self.ops = []  # (dst, "min"|"max", a, b)
        self.n_wires = n_inputs

    def _op(self, kind, a, b):
        d = self.n_wires
        self.n_wires += 1
        self.ops.append((d, kind, a, b))
        return d

    def mn(self, a, b):
        return self._op("min", a, b)

    def mx(self, a, b):
        return self._op("max", a, b)

    def ce(self, a, b):
        return self.mn(a, b), self.mx(a, b)

    # -- building blocks -------------------------------------------------
    def sort(self, wires):
        """Sorting network: a checked small network up to 7 inputs, else
        odd-even merge sort of the two halves."""
        w = list(wires)
        if len(w) in SORT_NETS:
            for i, j in SORT_NETS[len(w)]:
                w[i], w[j] = self.ce(w[i], w[j])
            return w
        half = len(w) // 2
        return self.oe_merge(self.sort(w[:half]), self.sort(w[half:]))

    def oe_merge(self, a, b):
        """Batcher's odd-even merge of two sorted lists of any lengths."""
        if not a:
            return list(b)
        if not b:
            return list(a)
        if len(a) == 1 and len(b) == 1:
            return list(self.ce(a[0], b[0]))
        ev = self.oe_merge(a[0::2], b[0::2])
        od = self.oe_merge(a[1::2], b[1::2])
        out = [ev[0]]
        i = 0
        while i < len(od):
            if i + 1 < len(ev):
                lo, hi = self.ce(od[i], ev[i + 1])
                out += [lo, hi]
            else:
                out.append(od[i])
            i += 1
        out += ev[len(od) + 1:]
        return out

    def select_rank(self, a, b, r):
        """r-th smallest (0-based) of sorted lists a and b:
        max over i of min(a[i], b[r - i]), out-of-range entries = +inf."""
        terms = []
        for i in range(max(0, r - len(b)), min(r, len(a)) + 1):
            j = r - i
            ai = a[i] if i < len(a) else None
            bj = b[j] if j < len(b) else None
            if ai is None and bj is None:
                continue
            terms.append(ai if bj is None else bj if ai is None else self.mn(ai, bj))
        acc = terms[0]
        for t in terms[1:]:
            acc = self.mx(acc, t)
        return acc

    # -- liveness --------------------------------------------------------
    def live_ops(self, outputs, start=0):
        live = set(outputs)
        keep = []
        for op in reversed(self.ops[start:]):
            if op[0] in live:
                keep.append(op)
                live.add(op[2])
                live.add(op[3])
        return keep[::-1]

    def prune(self, outputs):
        self.ops = self.live_ops(outputs)

    # -- evaluation (for self-tests) --------------------------------------
    def evaluate(self, inputs, outputs):
        """inputs: array (n_inputs, batch) -> array (len(outputs), batch)."""
        vals = {i: inputs[i] for i in range(self.n_inputs)}
        for d, kind, a, b in self.ops:
            vals[d] = np.minimum(vals[a], vals[b]) if kind == "min" else np.maximum(vals[a],
                                                                                    vals[b])
        return np.stack([vals[o] for o in outputs])


def merge_trimmed(net, a, b, lo, hi):
    """Sorted ranks lo..hi of a U b, using the cheaper of an odd-even merge
    and per-rank selection (counted by live operations)."""
    hi = min(hi, len(a) + len(b) - 1)
    lo = max(lo, 0)
    mark = len(net.ops)
    nw = net.n_wires
    m = net.oe_merge(a, b)[lo:hi + 1]
    cost_merge = len(net.live_ops(m, mark))
    ops_merge = net.ops[mark:]
    net.ops = net.ops[:mark]
    nw_merge = net.n_wires
    net.n_wires = max(nw, nw_merge)
    mark2 = len(net.ops)
    s = [net.select_rank(a, b, r) for r in range(lo, hi + 1)]
    cost_sel = len(net.live_ops(s, mark2))
    if cost_sel <= cost_merge:
        return s
    net.ops = net.ops[:mark2] + ops_merge
    return m


def median_of_sorted_lists(net, lists, n_total=None, med=None):
    """Median (rank med of n_total) of the union of sorted wire lists."""
    n = n_total if n_total is not None else sum(len(x) for x in lists)
    med = (n - 1) // 2 if med is None else med
    # each part: [wires, dropped_low, coverage]
    parts = [[list(x), 0, len(x)] for x in lists]
    while len(parts) > 1:
        parts.sort(key=lambda p: p[2])
        (wa, da, ca), (wb, db, cb) = parts[0], parts[1]
        cov = ca + cb
        drop = da + db
        t = n - cov
        lo_rank = max(0, med - t)
        hi_rank = min(med, cov - 1)
        if t == 0 and len(parts) == 2:
            return net.select_rank(wa, wb, med - drop)
        w = merge_trimmed(net, wa, wb, lo_rank - drop, hi_rank - drop)
        parts = parts[2:] + [[w, lo_rank, cov]]
    wires, drop, cov = parts[0]
    return wires[med - drop]


def line_median_net(k):
    """Median of k keys in a line (a row or a column of a window).  Five
    keys: the larger of the two pairs' minima and the smaller of their maxima
    bracket the median with the fifth key, whose median of three it is (10
    min/max; checked exhaustively).  Otherwise the middle output of a sorting
    network, pruned to what it needs."""
    net = Net(k)
    if k == 5:
        m1, x1 = net.ce(0, 1)
        m2, x2 = net.ce(2, 3)
        lo, hi = net.mx(m1, m2), net.mn(x1, x2)
        a, b = net.ce(4, lo)
        out = net.mx(a, net.mn(b, hi))
        return net, out
    out = net.sort(list(range(k)))[k // 2]
    net.prune([out])
    return net, out


def window_median_net(k):
    """Median of a k x k window, inputs v[r*k + c]."""
    net = Net(k * k)
    cols = [net.sort([r * k + c for r in range(k)]) for c in range(k)]
    out = median_of_sorted_lists(net, cols)
    net.prune([out])
    return net, out


def _trim_merge_all(net, parts, n, med, final):
    """Merge parts ([wires, dropped_low, coverage]) pairwise, smallest
    coverage first, trimming each partial result to the ranks that can still
    hold the median; with final, return the median wire."""
    parts = [list(p) for p in parts]
    while len(parts) > 1:
        parts.sort(key=lambda p: p[2])
        (wa, da, ca), (wb, db, cb) = parts[0], parts[1]
        cov = ca + cb
        drop = da + db
        t = n - cov
        if final and t == 0 and len(parts) == 2:
            return net.select_rank(wa, wb, med - drop)
        lo = max(0, med - t)
        hi = min(med, cov - 1)
        w = merge_trimmed(net, wa, wb, lo - drop, hi - drop)
        parts = parts[2:] + [[w, lo, cov]]
    if final:
        wires, drop, _ = parts[0]
        return wires[med - drop]
    return parts


def block_median_net(k, by, bx):
    """Medians of a by x bx block of k x k windows over a (by+k-1) x
    (bx+k-1) input patch (row-major).  The windows' common core is sorted
    and trimmed once; the block is split in halves recursively, each half
    adding the cells its windows share beyond the parent core, and each
    output finally adds its own remaining cells (every added set is sorted
    column by column first)."""
    r = k // 2
    n = k * k
    med = (n - 1) // 2
    H, W = by + 2 * r, bx + 2 * r
    net = Net(H * W)

    def window(oy, ox):
        return {(oy + dy, ox + dx) for dy in range(k) for dx in range(k)}

    def col_parts(cells):
        cols = {}
        for (y, x) in cells:
            cols.setdefault(x, []).append(y)
        return [[net.sort([y * W + x for y in sorted(ys)]), 0, len(ys)]
                for x, ys in sorted(cols.items())]

    outs = {}

    def node(cells_out, core_cells, core_parts):
        if len(cells_out) == 1:
            (oy, ox), = cells_out
            extra = window(oy, ox) - core_cells
            outs[(oy, ox)] = _trim_merge_all(net, core_parts + col_parts(extra), n, med, True)
            return
        ys = sorted({c[0] for c in cells_out})
        xs = sorted({c[1] for c in cells_out})
        if len(ys) >= len(xs):
            mid = ys[len(ys) // 2]
            halves = ([c for c in cells_out if c[0] < mid], [c for c in cells_out if c[0] >= mid])
        else:
            mid = xs[len(xs) // 2]
            halves = ([c for c in cells_out if c[1] < mid], [c for c in cells_out if c[1] >= mid])
        for half in halves:
            cc = set.intersection(*[window(*c) for c in half])
            parts = _trim_merge_all(net, core_parts + col_parts(cc - core_cells), n, med, False)
            node(half, cc, parts)

    cells = [(y, x) for y in range(by) for x in range(bx)]
    core = set.intersection(*[window(*c) for c in cells])
    node(cells, core, _trim_merge_all(net, col_parts(core), n, med, False))
    order = sorted(outs)
    out_wires = [outs[c] for c in order]
    net.prune(out_wires)
    return net, out_wires


def sort_all_net(n):
    net = Net(n)
    out = net.sort(list(range(n)))
    net.prune(out)
    return net, out


def med9_net():
    """3x3 median from sorted columns: med3(max of the column minima,
    med of the column medians, min of the column maxima)."""
    net = Net(9)
    cols = [net.sort([r * 3 + c for r in range(3)]) for c in range(3)]
    lo = net.mx(net.mx(cols[0][0], cols[1][0]), cols[2][0])
    md_a = cols[0][1]
    md_b = cols[1][1]
    md_c = cols[2][1]
    md = net.mx(net.mn(md_a, md_b), net.mn(net.mx(md_a, md_b), md_c))
    hi = net.mn(net.mn(cols[0][2], cols[1][2]), cols[2][2])
    out = net.mx(net.mn(lo, md), net.mn(net.mx(lo, md), hi))
    net.prune([out])
    return net, out


def emit_multi(net, outs, name, comment):
    lines = ["// %s" % comment, "// %d min/max operations." % len(net.ops),
             "__device__ __forceinline__ void %s(const int* v, int* o) {" % name]
    used = {a for _, _, a, b in net.ops} | {b for _, _, a, b in net.ops} | set(outs)
    for i in range(net.n_inputs):
        if i in used:
            lines.append("  const int w%d = v[%d];" % (i, i))
    for d, kind, a, b in net.ops:
        fn = "kmin" if kind == "min" else "kmax"
        lines.append("  const int w%d = %s(w%d, w%d);" % (d, fn, a, b))
    for j, wv in enumerate(outs):
        lines.append("  o[%d] = w%d;" % (j, wv))
    lines.append("}")
    return "\n".join(lines)


def emit(net, out, name, comment):
    lines = ["// %s" % comment, "// %d min/max operations." % len(net.ops),
             "__device__ __forceinline__ int %s(const int* v) {" % name]
    for i in range(net.n_inputs):
        lines.append("  const int w%d = v[%d];" % (i, i))
    for d, kind, a, b in net.ops:
        fn = "kmin" if kind == "min" else "kmax"
        lines.append("  const int w%d = %s(w%d, w%d);" % (d, fn, a, b))
    lines.append("  return w%d;" % out)
    lines.append("}")
    return "\n".join(lines)


def _check_sort_nets():
    for n, comps in SORT_NETS.items():
        for bits in itertools.product((0, 1), repeat=n):
            v = list(bits)
            for i, j in comps:
                if v[i] > v[j]:
                    v[i], v[j] = v[j], v[i]
            assert v == sorted(v), ("sorting network", n, bits)


def _check_median(net, out, n, exhaustive):
    med = (n - 1) // 2
    if exhaustive:
        # every 0-1 input: by the 0-1 principle this proves the network
        codes = np.arange(1 << n, dtype=np.int64)
        inputs = ((codes[None, :] >> np.arange(n)[:, None]) & 1).astype(np.int32)
        got = net.evaluate(inputs, [out])[0]
        ref = (inputs.sum(axis=0) > med).astype(np.int32)
        assert np.array_equal(got, ref), "0-1 check failed"
    g = np.random.default_rng(1)
    for hi in (2, 5, 50, 1 << 30):
        inputs = g.integers(-hi, hi, size=(n, 20000)).astype(np.int64)
        got = net.evaluate(inputs, [out])[0]
        ref = np.sort(inputs, axis=0)[med]
        assert np.array_equal(got, ref), "random check failed"


def _check_block(net, outs, k, by, bx):
    """Random inputs with many ties: every output against a sort of its
    window."""
    r = k // 2
    H, W = by + 2 * r, bx + 2 * r
    g = np.random.default_rng(2)
    for hi in (2, 4, 30, 1 << 30):
        x = g.integers(-hi, hi, size=(H * W, 20000)).astype(np.int64)
        got = net.evaluate(x, outs)
        X = x.reshape(H, W, -1)
        j = 0
        for oy in range(by):
            for ox in range(bx):
                ref = np.sort(X[oy:oy + k, ox:ox + k].reshape(k * k, -1), axis=0)[(k * k - 1) // 2]
                assert np.array_equal(got[j], ref), ("block", k, by, bx, oy, ox)
                j += 1


def _check_sort_prefix(net, outs, n):
    g = np.random.default_rng(4)
    k = len(outs)
    for hi in (2, 5, 1 << 30):
        x = g.integers(-hi, hi, size=(n, 20000)).astype(np.int64)
        assert np.array_equal(net.evaluate(x, outs), np.sort(x, axis=0)[:k]), "sort prefix"


def _check_sort(net, outs, n):
    g = np.random.default_rng(3)
    for hi in (2, 5, 1 << 30):
        x = g.integers(-hi, hi, size=(n, 20000)).astype(np.int64)
        assert np.array_equal(net.evaluate(x, outs), np.sort(x, axis=0)), "sort"


def build_all(check=False):
    if check:
        _check_sort_nets()
    parts = []
    n9, o9 = med9_net()
    n25, o25 = window_median_net(5)
    n49, o49 = window_median_net(7)
    nb, ob = block_median_net(5, 2, 2)
    nq, oq = block_median_net(5, 4, 2)
    ns, os_ = sort_all_net(25)
    nl, ol = sort_all_net(25)
    nl.prune(ol[:13])
    ol = ol[:13]
    lines = {k: line_median_net(k) for k in (5, 7)}
    if check:
        for k, (nk, ok) in lines.items():
            _check_median(nk, ok, k, exhaustive=True)
        _check_median(n9, o9, 9, exhaustive=True)
        _check_median(n25, o25, 25, exhaustive=True)
        _check_median(n49, o49, 49, exhaustive=False)
        _check_block(nb, ob, 5, 2, 2)
        _check_block(nq, oq, 5, 4, 2)
        _check_sort(ns, os_, 25)
        _check_sort_prefix(nl, ol, 25)
    parts.append(emit(n9, o9, "med9", "Median of 9 keys (3x3 window, row-major)."))
    parts.append(emit(n25, o25, "med25", "Median of 25 keys (5x5 window, row-major)."))
    parts.append(emit(n49, o49, "med49", "Median of 49 keys (7x7 window, row-major)."))
    parts.append(emit_multi(nb, ob, "med25_2x2",
                            "5x5 medians of a 2x2 block of windows over a 6x6 patch "
                            "(row-major); o = {(0,0), (0,1), (1,0), (1,1)}."))
    parts.append(emit_multi(nq, oq, "med25_4x2",
                            "5x5 medians of a 4x2 block of windows over an 8x6 patch "
                            "(row-major); o[2 * row + col]."))
    parts.append(emit_multi(ns, os_, "sort25", "All 25 keys in ascending order."))
    parts.append(emit_multi(nl, ol, "sort25_lo13",
                            "The 13 smallest of 25 keys in ascending order (ranks 0..12)."))
    for k, (nk, ok) in lines.items():
        parts.append(emit(nk, ok, "medline%d" % k,
                          "Median of %d keys in a line (the separable median's passes)." % k))
    return parts, dict(med9=len(n9.ops), med25=len(n25.ops), med49=len(n49.ops),
                       med25_2x2=len(nb.ops), med25_4x2=len(nq.ops), sort25=len(ns.ops), sort25_lo13=len(nl.ops),
                       medline5=len(lines[5][0].ops), medline7=len(lines[7][0].ops))


HEADER = """// Generated by gen_median_net.py -- do not edit.
// Selection networks over 32-bit keys whose signed order is the float order.
#pragma once
__device__ __forceinline__ int kmin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int kmax(int a, int b) { return a > b ? a : b; }
"""


def main(argv):
    check = "--check" in argv
    args = [a for a in argv if not a.startswith("--")]
    parts, counts = build_all(check=check)
    text = HEADER + "\n" + "\n\n".join(parts) + "\n"
    if args:
        with open(args[0], "w") as f:
            f.write(text)
    print("networks:", counts, "(checked)" if check else "")


if __name__ == "__main__":
    main(sys.argv[1:])
