"""Host logic of the benchmark's batch pipeline: the enqueue order is free of hazards.

The benchmark enqueues, per batch i, a phase space `ps` (writes the event buffer
i mod B and reads the Vegas grid), a matrix element `me` (reads the event buffer,
writes its |M|^2 array) and a Vegas call `vg` (reads both; the last batch of a
Vegas iteration also rewrites the grid).  B = 1 buffer with one stream, 2 with
more.  Streams: `ps` on a side stream (2 or 3 streams), `me` on the main stream,
`vg` on a third stream (3 streams) or the main one.  Ordering comes from FIFO
order on each stream and from event waits: `ps` waits for the `free` event of
its buffer (recorded by each `vg` of that buffer) and, when it opens an
iteration, for `grid_done` (recorded by the refining `vg`); `me` waits for
`ready` (recorded by `ps`); `vg` waits for `computed` (recorded by `me`).  A
wait sees the event's latest record at the time it is enqueued.  From that
model the test builds the happens-before relation of an enqueue order and
checks that every batch reads its own phase space, that no matrix element
overwrites a result before its Vegas call has read it, that the Vegas calls
stay in batch order, and that every batch sees the grid of the previous
iteration.
"""
import pytest

import bench

ITER = bench.BATCHES_PER_ITER


def stream_of(kind, streams):
    if kind == 'ps':
        return 'side' if streams >= 2 else 'main'
    if kind == 'vg':
        return 'vg' if streams == 3 else 'main'
    return 'main'


def happens_before(order, streams):
    """Transitive happens-before over the ops of `order` as a set of (a, b) pairs."""
    nbuf = 1 if streams == 1 else 2
    edges = set()
    last_on = {}
    last_rec = {}                                   # event name -> op that last recorded it
    waits = {'ps': lambda i: [('free', i % nbuf)] + ([('grid',)] if i % ITER == 0 else []),
             'me': lambda i: [('ready', i % nbuf)],
             'vg': lambda i: [('computed', i % nbuf)]}
    records = {'ps': lambda i: [('ready', i % nbuf)],
               'me': lambda i: [('computed', i % nbuf)],
               'vg': lambda i: [('free', i % nbuf)] + ([('grid',)] if (i + 1) % ITER == 0 else [])}
    for op in order:
        kind, i = op
        s = stream_of(kind, streams)
        if s in last_on:
            edges.add((last_on[s], op))
        last_on[s] = op
        for ev in waits[kind](i):
            if ev in last_rec:
                edges.add((last_rec[ev], op))
        for ev in records[kind](i):
            last_rec[ev] = op
    hb = set(edges)
    nodes = list(order)
    for k in nodes:                                 # Floyd-Warshall closure
        for a in nodes:
            if (a, k) in hb:
                for b in nodes:
                    if (k, b) in hb:
                        hb.add((a, b))
    return hb


def hazards(order, streams):
    nbuf = 1 if streams == 1 else 2
    hb = happens_before(order, streams)
    ops = set(order)
    batches = sorted({i for _, i in order})
    bad = []
    for i in batches:
        ps, me, vg = ('ps', i), ('me', i), ('vg', i)
        if (ps, me) not in hb or (me, vg) not in hb:
            bad.append(f'batch {i}: phase space, matrix element and Vegas call out of order')
        for j in batches:
            if j == i or j % nbuf != i % nbuf:
                continue
            # the event buffer stays intact from ps(i) until vg(i) has read it
            if not ((('ps', j), ps) in hb or (vg, ('ps', j)) in hb):
                bad.append(f'ps {j} may overwrite the buffer of batch {i}')
            # the |M|^2 array stays intact from me(i) until vg(i) has read it
            if not ((('me', j), me) in hb or (vg, ('me', j)) in hb):
                bad.append(f'me {j} may overwrite the matrix elements of batch {i}')
        if ('vg', i + 1) in ops and (vg, ('vg', i + 1)) not in hb:
            bad.append(f'Vegas calls {i} and {i + 1} may run out of order')
        it = i // ITER
        refine_before = ('vg', it * ITER - 1)
        if refine_before in ops and (refine_before, ps) not in hb:
            bad.append(f'ps {i} may read the grid before the refine of batch {it * ITER - 1}')
        refine_after = ('vg', it * ITER + ITER - 1)
        if refine_after in ops and (ps, refine_after) not in hb:
            bad.append(f'ps {i} may read the grid after the refine of batch {it * ITER + ITER - 1}')
    return bad


@pytest.mark.parametrize('streams', [1, 2, 3])
@pytest.mark.parametrize('first,count', [(0, 1), (0, 2), (1, 18), (15, 3), (16, 17), (3, 40)])
def test_enqueue_order_has_no_hazard(streams, first, count):
    order = bench.enqueue_order(first, count, streams)
    assert sorted(order) == sorted([(k, i) for i in range(first, first + count) for k in ('ps', 'me', 'vg')])
    assert hazards(order, streams) == []


@pytest.mark.parametrize('streams', [2, 3])
def test_pipeline_overlaps(streams):
    """ps(i+1) is unordered with me(i) except where i+1 opens an iteration; with three
    streams vg(i) is also unordered with me(i+1)."""
    first, count = 1, 40
    order = bench.enqueue_order(first, count, streams)
    hb = happens_before(order, streams)

    def ordered(a, b):
        return (a, b) in hb or (b, a) in hb
    for i in range(first, first + count - 1):
        assert ordered(('me', i), ('ps', i + 1)) == ((i + 1) % ITER == 0), i
        assert ordered(('vg', i), ('me', i + 1)) == (streams == 2 or (i + 1) % ITER == 0), i


def _bad_order(first, count):
    order = [('ps', first)]
    for i in range(first, first + count):
        if i + 1 < first + count:
            order.append(('ps', i + 1))
        order += [('me', i), ('vg', i)]
    return order


def test_checker_flags_look_ahead_on_one_buffer():
    """Phase space of i+1 enqueued before the rest of i on a single buffer is caught."""
    order = _bad_order(1, 5)
    assert hazards(order, 1)
    assert not hazards(order, 2)


def test_checker_flags_grid_read_before_refine():
    """Phase space of an iteration's first batch enqueued before the previous refine is caught."""
    bad = hazards(_bad_order(ITER - 2, 4), 3)
    assert any('grid' in b for b in bad), bad


def test_checker_flags_missing_vegas_wait():
    """A Vegas call enqueued before its matrix element is caught."""
    order = bench.enqueue_order(1, 6, 3)
    k = order.index(('vg', 3))
    order.insert(order.index(('me', 3)), order.pop(k))
    bad = hazards(order, 3)
    assert any('out of order' in b for b in bad), bad
