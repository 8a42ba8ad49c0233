"""Host logic of the benchmark's batch pipeline: the enqueue order is free of hazards.

The benchmark enqueues, per batch i, a phase space `ps` (writes buffer i mod S,
reads the Vegas grid) and a `rest` (matrix element and Vegas call: reads the
buffer; the last batch of a Vegas iteration also rewrites the grid).  With S = 2
the `ps` ops go to a second stream.  Ordering comes from FIFO order on each
stream and from event waits: `ps` waits for the `free` event of its buffer
(recorded by each `rest` of that buffer) and, when it opens an iteration, for
`grid_done` (recorded by the refining `rest`); `rest` waits for the `ready` event
of its buffer (recorded by each `ps` of that buffer).  A wait sees the event's
latest record at the time it is enqueued.  From that model the test builds the
happens-before relation of an enqueue order and checks that every batch reads
its own phase space and the grid of the previous iteration.
"""
import pytest

import bench

ITER = bench.BATCHES_PER_ITER


def happens_before(order, streams):
    """Transitive happens-before over the ops of `order` as a set of (a, b) pairs."""
    stream_of = {'ps': 'side' if streams > 1 else 'main', 'rest': 'main'}
    edges = set()
    last_on = {}
    last_rec = {}                                   # event name -> op that last recorded it
    for op in order:
        kind, i = op
        s = stream_of[kind]
        if s in last_on:
            edges.add((last_on[s], op))
        last_on[s] = op
        buf = i % streams
        if kind == 'ps':
            waits = [('free', buf)] + ([('grid',)] if i % ITER == 0 else [])
            for ev in waits:
                if ev in last_rec:
                    edges.add((last_rec[ev], op))
            last_rec[('ready', buf)] = op
        else:
            if ('ready', buf) in last_rec:
                edges.add((last_rec[('ready', buf)], op))
            last_rec[('free', buf)] = op
            if (i + 1) % ITER == 0:
                last_rec[('grid',)] = op
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
    hb = happens_before(order, streams)
    ops = set(order)
    batches = sorted({i for _, i in order})
    bad = []
    for i in batches:
        ps, rest = ('ps', i), ('rest', i)
        if (ps, rest) not in hb:
            bad.append(f'rest {i} not after ps {i}')
        for j in batches:
            if j != i and j % streams == i % streams:
                other = ('ps', j)
                # every other write of the buffer is before ps(i) or after rest(i)
                if not ((other, ps) in hb or (rest, other) in hb):
                    bad.append(f'ps {j} may overwrite the buffer of batch {i}')
        it = i // ITER
        refine_before = ('rest', it * ITER - 1)
        if refine_before in ops and (refine_before, ps) not in hb:
            bad.append(f'ps {i} may read the grid before the refine of batch {it * ITER - 1}')
        refine_after = ('rest', it * ITER + ITER - 1)
        if refine_after in ops and (ps, refine_after) not in hb:
            bad.append(f'ps {i} may read the grid after the refine of batch {it * ITER + ITER - 1}')
    return bad


@pytest.mark.parametrize('streams', [1, 2])
@pytest.mark.parametrize('first,count', [(0, 1), (0, 2), (1, 18), (15, 3), (16, 17), (3, 40)])
def test_enqueue_order_has_no_hazard(streams, first, count):
    order = bench.enqueue_order(first, count, streams)
    assert sorted(order) == sorted([('ps', i) for i in range(first, first + count)] +
                                   [('rest', i) for i in range(first, first + count)])
    assert hazards(order, streams) == []


def test_two_streams_overlap_phase_space_with_matrix_element():
    """With two streams, ps(i+1) is unordered with rest(i) except where i+1 opens an iteration."""
    first, count = 1, 40
    order = bench.enqueue_order(first, count, 2)
    hb = happens_before(order, 2)
    for i in range(first, first + count - 1):
        ordered = (('rest', i), ('ps', i + 1)) in hb or (('ps', i + 1), ('rest', i)) in hb
        assert ordered == ((i + 1) % ITER == 0), i


def test_checker_flags_look_ahead_on_one_buffer():
    """Phase space of i+1 enqueued before the rest of i on a single buffer is caught."""
    first, count = 1, 5
    order = [('ps', first)]
    for i in range(first, first + count):
        if i + 1 < first + count:
            order.append(('ps', i + 1))
        order.append(('rest', i))
    assert hazards(order, 1)
    assert not hazards(order, 2)


def test_checker_flags_grid_read_before_refine():
    """Phase space of an iteration's first batch enqueued before the previous refine is caught."""
    first, count = ITER - 2, 4
    order = [('ps', first)]
    for i in range(first, first + count):
        if i + 1 < first + count:
            order.append(('ps', i + 1))
        order.append(('rest', i))
    bad = hazards(order, 2)
    assert any('grid' in b for b in bad), bad
