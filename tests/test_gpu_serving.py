"""GPU parity of the task-list entry point and the request server: every
request's coreness is the oracle's, and the same whether the graph is
decomposed alone or in a mix of requests that are admitted, batched and run
concurrently by the server."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2402_15253_amd as pico

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool():
    """A device-resident pool of graphs of mixed size (some above the LDS
    tier, some empty or edgeless) with their oracle coreness."""
    b = gg.mixed_batch(40, 2, 40_000, seed=77, device="cuda")
    graphs = []
    for g in range(b.num_graphs):
        x0, x1 = int(b.vptr[g]), int(b.vptr[g + 1])
        off = b.offsets[x0:x1 + 1]  # positions into b.cols, not starting at 0
        m = int(off[-1] - off[0]) if x1 > x0 else 0
        cpu = b.graph(g)
        want = oracle.bz_coreness(cpu.offsets.cpu(), cpu.cols.cpu())
        graphs.append({"off": off, "n": x1 - x0, "m": m, "want": want})
    return b, graphs


def _scratch(n, m, algo):
    nbytes = pico.pico_task_scratch_bytes(n, m, algo)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("algo", ["peelone", "histocore", "auto"])
def test_tasks_match_oracle(pool, algo):
    b, graphs = pool
    code = pico.BATCH_ALGOS[algo]
    keep, tasks = [], []
    order = sorted(range(len(graphs)), key=lambda i: -graphs[i]["n"])
    for i in order:
        g = graphs[i]
        out = torch.full((max(g["n"], 1),), -1, dtype=torch.int32, device="cuda")
        s = _scratch(g["n"], g["m"], code)
        keep.append((i, out, s))
        tasks.append(pico.Task(g["off"].data_ptr(), b.cols.data_ptr(), g["n"], g["m"], out.data_ptr(),
                               s.data_ptr(), s.numel()))
    wsb = pico.pico_tasks_workspace_bytes(len(tasks))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st = pico.BatchStats()
    rc = pico.pico_coreness_tasks(tasks, code, pico.BatchTune(), ws, wsb, st)
    assert rc == pico.PICO_OK, pico.pico_last_error()
    print(f"{algo} stats={st.as_dict()}", flush=True)
    for i, out, _ in keep:
        g = graphs[i]
        assert np.array_equal(out[:g["n"]].cpu().numpy(), g["want"]), f"graph {i} n={g['n']}"
    assert st.graphs == len(tasks) and st.lds_graphs > 0 and st.lds_graphs < len(tasks)
    rc, words = pico.batch_status(ws, len(tasks))
    assert rc == pico.PICO_OK and (words == 0).all()


@pytest.mark.parametrize("algo", ["peelone", "histocore", "auto"])
def test_server_alone_vs_mix(pool, algo):
    """Requests arrive in bursts while earlier ones run; the arena admits only
    part of them at a time, up to three launches are in flight, and small
    class bounds spread the pool over all three size classes.  Each result
    equals the graph's result alone (the plain single-graph call) and the
    oracle's."""
    b, graphs = pool
    code = pico.BATCH_ALGOS[algo]
    alone = []
    for g in graphs:
        if g["n"] == 0:
            alone.append(np.zeros(0, dtype=np.int32))
            continue
        off = (g["off"] - g["off"][0]).contiguous()
        e0 = int(g["off"][0])
        core = pico.coreness(off, b.cols[e0:e0 + g["m"]], algo)
        alone.append(core.cpu().numpy())
    for g, a in zip(graphs, alone):
        assert np.array_equal(a, g["want"])
    need = [pico.pico_task_scratch_bytes(g["n"], g["m"], code) for g in graphs]
    arena = max(3 * max(need), 1 << 20)  # well below the sum over all requests
    srv = pico.Server(algo, arena_bytes=arena, max_inflight=3, max_tasks_per_launch=16,
                      class_bounds=(2000, 12000), max_large_slots=1)
    rng = np.random.default_rng(5)
    R = 300
    pick = rng.integers(0, len(graphs), R)
    sizes = [graphs[p]["n"] for p in pick]
    base = np.concatenate([[0], np.cumsum(sizes)])
    out = torch.full((int(base[-1]) + 1,), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # the server runs on its own streams
    done, r, peak_wait = {}, 0, 0
    while len(done) < R:
        burst = int(rng.integers(1, 12))
        for _ in range(burst):
            if r == R:
                break
            g = graphs[pick[r]]
            srv.submit_ptrs(g["off"].data_ptr(), b.cols.data_ptr(), g["n"], g["m"],
                            out.data_ptr() + 4 * int(base[r]), r)
            r += 1
        for c in srv.progress():
            assert c.status == pico.PICO_OK
            assert c.tag not in done
            assert c.t_submit_ns <= c.t_launch_ns <= c.t_done_ns
            done[c.tag] = c
        peak_wait = max(peak_wait, srv.status()["waiting"])
    st = srv.status()
    srv.close()
    assert st["completed"] == R and st["arena_used"] == 0 and st["waiting"] == 0
    assert st["launches"] > 1
    print(f"{algo}: {st} peak waiting {peak_wait}", flush=True)
    got = out.cpu().numpy()
    for i in range(R):
        p = pick[i]
        assert np.array_equal(got[base[i]:base[i + 1]], alone[p]), f"request {i} graph {p}"


def test_server_rejects_what_never_fits(pool):
    b, graphs = pool
    g = max(graphs, key=lambda g: g["n"])
    srv = pico.Server("peelone", arena_bytes=1 << 16, max_inflight=1, max_tasks_per_launch=4)
    out = torch.empty(g["n"], dtype=torch.int32, device="cuda")
    with pytest.raises(pico.PicoError) as e:
        srv.submit(g["off"], b.cols, g["n"], g["m"], out, 0)
    assert e.value.status == pico.PICO_ENOMEM
    srv.close()


@pytest.mark.skip(reason="persistent request-queue kernel (a kernel polling a request ring in pinned "
                         "host memory and writing completion words there) faulted the GPU twice "
                         "on its first requests; switched off (the server uses launch slots)")
def test_persistent_queue_server_alone_vs_mix():
    """Placeholder for the persistent-queue form of the server: the same
    alone-versus-mix check as test_server_alone_vs_mix, with one kernel
    instance taking requests from a host ring."""
    raise AssertionError("persistent queue mode is switched off")


@pytest.mark.parametrize("algo", ["peelone", "histocore"])
def test_helped_tasks_repeatable(algo):
    """Large tasks decomposed with 32 helpers each, next to small ones,
    repeated: every run equals the single-graph result.  (Helpers count a
    chunk done only after every wave of the workgroup has its stores and
    atomics performed.)"""
    b = gg.mixed_batch(6, 150_000, 300_000, seed=91, device="cuda")
    code = pico.ALGOS[algo]
    alone, keep, tasks = [], [], []
    for g in range(b.num_graphs):
        x0, x1 = int(b.vptr[g]), int(b.vptr[g + 1])
        off = b.offsets[x0:x1 + 1]
        n, m = x1 - x0, int(off[-1] - off[0])
        e0 = int(off[0])
        alone.append(pico.coreness((off - e0).contiguous(), b.cols[e0:e0 + m], "peelone").cpu().numpy())
        print(f"case {algo} graph {g} n={n} m={m}", flush=True)
        out = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        s = _scratch(n, m, code)
        keep.append((out, s))
        tasks.append(pico.Task(off.data_ptr(), b.cols.data_ptr(), n, m, out.data_ptr(), s.data_ptr(),
                               s.numel()))
    order = sorted(range(len(tasks)), key=lambda i: -tasks[i].n)
    wsb = pico.pico_tasks_workspace_bytes(len(tasks))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    for rep in range(4):
        st = pico.BatchStats()
        rc = pico.pico_coreness_tasks([tasks[i] for i in order], code, pico.BatchTune(-1, 0, 0, 32768),
                                      ws, wsb, st)
        assert rc == pico.PICO_OK, pico.pico_last_error()
        assert st.helped_graphs == len(tasks) and st.help_chunks > 0
        for i in range(len(tasks)):
            assert np.array_equal(keep[i][0].cpu().numpy(), alone[i]), f"rep {rep} graph {i}"


@pytest.mark.parametrize("algo", ["peelone", "auto"])
def test_server_trace_every_class_against_oracle(algo):
    """A trace of 600 requests over a pool whose graphs reach every size class
    (below 16,384 vertices, below 131,072, above) with the library's class
    bounds, helpers for the large ones and four launch slots: every request's
    output is compared with the oracle, vertex by vertex, and every
    completion reads PICO_OK."""
    b = gg.mixed_batch(30, 300, 240_000, seed=2000, device="cuda")
    graphs = []
    for g in range(b.num_graphs):
        x0, x1 = int(b.vptr[g]), int(b.vptr[g + 1])
        off = b.offsets[x0:x1 + 1]
        m = int(off[-1] - off[0]) if x1 > x0 else 0
        cpu = b.graph(g)
        graphs.append({"off": off, "n": x1 - x0, "m": m,
                       "want": oracle.bz_coreness(cpu.offsets.cpu(), cpu.cols.cpu())})
    sizes = np.array([g["n"] for g in graphs])
    assert (sizes < 16384).any() and ((sizes >= 16384) & (sizes < 131072)).any() and (sizes >= 131072).any()
    code = pico.BATCH_ALGOS[algo]
    need = sum(pico.pico_task_scratch_bytes(g["n"], g["m"], code) for g in graphs)
    srv = pico.Server(algo, arena_bytes=max(need, 1 << 20), max_inflight=4, max_tasks_per_launch=64)
    rng = np.random.default_rng(11)
    R = 600
    pick = rng.integers(0, len(graphs), R)
    base = np.concatenate([[0], np.cumsum(sizes[pick])])
    out = torch.full((int(base[-1]) + 1,), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    done, r = 0, 0
    while done < R:
        for _ in range(int(rng.integers(1, 16))):
            if r == R:
                break
            g = graphs[pick[r]]
            srv.submit_ptrs(g["off"].data_ptr(), b.cols.data_ptr(), g["n"], g["m"],
                            out.data_ptr() + 4 * int(base[r]), r)
            r += 1
        for c in srv.progress():
            assert c.status == pico.PICO_OK, c.tag
            done += 1
    st = srv.status()
    srv.close()
    print(f"{algo}: {st}", flush=True)
    got = out.cpu().numpy()
    for i in range(R):
        assert np.array_equal(got[base[i]:base[i + 1]], graphs[pick[i]]["want"]), f"request {i} graph {pick[i]}"
