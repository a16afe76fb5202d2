"""The oracle's particle arrays reach its C routines in [7][n] row-major
layout whatever layout they are handed in: an id-sorted copy (which numpy
lays out column-major) steps and estimates exactly like the same values in
row-major order."""
import numpy as np

import oracle as O
from synth import configs as CF


def test_column_major_state_steps_like_row_major():
    w = CF.periodic_square(n=8, ppe=20)
    o = O.Oracle(w.mesh, w.params)
    o.seed(w.seed)
    o.run(w.dt, 2)
    order = np.argsort(-o.id.astype(np.int64), kind="stable")
    st, el, pid, stats = o.state[:, order], o.elem[order], o.id[order], o.stats.copy()
    assert st.flags["F_CONTIGUOUS"] and not st.flags["C_CONTIGUOUS"]
    runs = []
    for state in (st, np.ascontiguousarray(st)):
        a = O.Oracle(w.mesh, w.params)
        a.seed(w.seed)
        a.state, a.elem, a.id = state, el.copy(), pid.copy()
        a.step_index = 2
        a.set_stats(stats)
        a.step(w.dt)
        runs.append((a.state.copy(), a.elem.copy(), a.stats.copy()))
    for x, y in zip(runs[0], runs[1]):
        assert np.array_equal(x, y)
