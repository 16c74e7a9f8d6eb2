"""Brute-force transfer counts of the resident loop nests (test infrastructure only).

Independent check of the data-movement model: the loop nests of Sec. 2.2
(Resident C, A, B) are run element by element, and every access goes through
a fast memory of M elements with Belady's optimal replacement (evict the
element whose next use is farthest).  Counted: reads from slow memory per
operand (misses), and writes to slow memory (evictions of modified C entries
plus the final flush).  With beta == 0 the first touch of a C entry is a
write without a read.

Capacity used: the resident block plus one streamed row and column (the
footnote of Sec. 2.2.1: m_c, n_c slightly below sqrt(M) leave room for them).
"""
import heapq


def _trace_resident_c(m, n, k, mc, nc):
    for ib in range(0, m, mc):
        for jb in range(0, n, nc):
            for p in range(k):                      # rank-1 updates
                for i in range(ib, min(ib + mc, m)):
                    yield ("A", i, p)
                    for j in range(jb, min(jb + nc, n)):
                        yield ("B", p, j)
                        yield ("C", i, j)


def _trace_resident_a(m, n, k, mc, kc):
    for ib in range(0, m, mc):
        for pb in range(0, k, kc):
            for j in range(n):                      # matrix-vector products
                for i in range(ib, min(ib + mc, m)):
                    for p in range(pb, min(pb + kc, k)):
                        yield ("A", i, p)
                        yield ("B", p, j)
                    yield ("C", i, j)


def _trace_resident_b(m, n, k, kc, nc):
    for jb in range(0, n, nc):
        for pb in range(0, k, kc):
            for i in range(m):                      # vector-matrix products
                for j in range(jb, min(jb + nc, n)):
                    for p in range(pb, min(pb + kc, k)):
                        yield ("B", p, j)
                        yield ("A", i, p)
                    yield ("C", i, j)


def simulate(resident, m, n, k, b1, b2, beta=1.0):
    """Counts for Resident C (b1, b2 = mc, nc), A (mc, kc) or B (kc, nc)."""
    if resident == "C":
        trace = list(_trace_resident_c(m, n, k, b1, b2))
        cap = b1 * b2 + b1 + b2
    elif resident == "A":
        trace = list(_trace_resident_a(m, n, k, b1, b2))
        cap = b1 * b2 + b2 + b1
    elif resident == "B":
        trace = list(_trace_resident_b(m, n, k, b1, b2))
        cap = b1 * b2 + b1 + b2
    else:
        raise ValueError(resident)
    # next-use index of every access
    nxt = [0] * len(trace)
    last = {}
    for t in range(len(trace) - 1, -1, -1):
        nxt[t] = last.get(trace[t], float("inf"))
        last[trace[t]] = t
    cache = {}          # element -> next use
    heap = []           # (-next_use, element) lazy max-heap
    dirty = set()
    touched_c = set()
    reads = {"A": 0, "B": 0, "C": 0}
    writes = 0
    for t, e in enumerate(trace):
        if e not in cache:
            if e[0] == "C" and e not in touched_c and beta == 0.0:
                pass                                # first touch overwrites: no read
            else:
                reads[e[0]] += 1
            while len(cache) >= cap:
                negu, victim = heapq.heappop(heap)
                if victim in cache and cache[victim] == -negu:
                    del cache[victim]
                    if victim in dirty:
                        writes += 1
                        dirty.discard(victim)
        cache[e] = nxt[t]
        heapq.heappush(heap, (-nxt[t], e))
        if e[0] == "C":
            touched_c.add(e)
            dirty.add(e)
    writes += len(dirty)
    return {"a_reads": reads["A"], "b_reads": reads["B"], "c_reads": reads["C"], "c_writes": writes}


def simulate_lru(resident, m, n, k, b1, b2, beta=1.0, panels=2):
    """Same loop nests through an LRU fast memory holding the resident block
    plus `panels` streamed rows and columns (Sec. 4.1: with LRU the panels a
    loop exposes must fit beside the block)."""
    from collections import OrderedDict
    if resident == "C":
        trace = _trace_resident_c(m, n, k, b1, b2)
        cap = b1 * b2 + panels * (b1 + b2)
    elif resident == "A":
        trace = _trace_resident_a(m, n, k, b1, b2)
        cap = b1 * b2 + panels * (b2 + b1)
    elif resident == "B":
        trace = _trace_resident_b(m, n, k, b1, b2)
        cap = b1 * b2 + panels * (b1 + b2)
    else:
        raise ValueError(resident)
    cache = OrderedDict()   # element -> dirty
    touched_c = set()
    reads = {"A": 0, "B": 0, "C": 0}
    writes = 0
    for e in trace:
        if e in cache:
            cache.move_to_end(e)
        else:
            if not (e[0] == "C" and e not in touched_c and beta == 0.0):
                reads[e[0]] += 1
            if len(cache) >= cap:
                _, d = cache.popitem(last=False)
                writes += 1 if d else 0
            cache[e] = False
        if e[0] == "C":
            touched_c.add(e)
            cache[e] = True
    writes += sum(1 for d in cache.values() if d)
    return {"a_reads": reads["A"], "b_reads": reads["B"], "c_reads": reads["C"], "c_writes": writes}
