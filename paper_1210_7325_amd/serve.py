"""Continuous-batching server for GWAS jobs (several cohorts on one GPU).

Jobs (a cohort: its own n, M, X_L, y, and m genotype problems) arrive over
time.  The scheduler admits them in arrival order while their device
footprint fits the HBM budget (each admitted job keeps its factor of M and
its whitened fixed part resident until it finishes), and every round it
takes the next block of problems from each active job and solves all of
them with ONE launch of the whitening kernel and one of the assembly/solve
kernel (gls_solve_multi).  Jobs that arrive while others run are admitted as
soon as memory frees up and their blocks join the next round, so the work of
different jobs overlaps on the device.  Rounds are queued four deep and
alternate over two compute streams, so the device never waits for the host
between rounds and the next round's work-groups take the compute units that
the previous round's last slabs leave free (rounds overlap on the device as
items of one persistent launch would, without a device-wide barrier between
them).

Each job's blocks are sized so that all items of a round cost about the
same (block ~ n^-2), and a job's results do not depend on what it was
batched with (bitwise).

A job's genotypes reach the device through host memory, as they would from
a job's files: for every round the executor produces the items' genotype
blocks on the host (the C generator stands in for the job's source) into a
pinned staging slot, copies the slot to the device on a copy stream, and
the compute stream waits for that copy before the round's launches; with
three slots, the host production and the copy of the next round overlap the
device work of the previous ones, and job latency includes the ingestion.

The scheduler is plain Python logic over an executor interface; `GpuExecutor`
drives libgls.so, and tests drive the scheduler with a fake executor.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import datagen as dg


@dataclasses.dataclass
class Job:
    id: int
    arrival: float          # seconds after the start of the run
    n: int
    p: int                  # p_L = p - 1 (intercept + covariates), p_R = 1
    m: int
    h: float
    seed: int
    # filled in by the scheduler
    block: int = 0          # problems per item when the device is shared
    max_block: int = 0      # largest item (when few jobs share the device)
    state: str = "pending"  # pending -> active -> done | failed
    admitted: Optional[float] = None
    finished: Optional[float] = None
    submitted: int = 0      # problems handed to rounds
    completed: int = 0      # problems whose round has finished
    error: Optional[str] = None

    @property
    def p_L(self) -> int:
        return self.p - 1

    def workload(self) -> dg.Workload:
        return dg.Workload(f"job{self.id}", n=self.n, p_L=self.p - 1, p_R=1, t=1, m=self.m,
                           block=self.block or 4096, q=2 * self.n, h=self.h, seed=self.seed)


def job_block(n: int, ref_n: int = 10_000, ref_block: int = 4096) -> int:
    """Problems per round for a cohort of n individuals: equal work per item
    (the whitening costs n^2 per problem), a multiple of 64, in [256, 65536]."""
    b = ref_block * (ref_n / n) ** 2
    return int(min(65536, max(256, round(b / 64) * 64)))


def make_jobs(count: int, rate: float, seed: int = dg.MASTER_SEED + 3,
              n_choices: Sequence[int] = (1500, 4000, 10000, 20000),
              p_range=(4, 20), m_range=(1e5, 1e7), h_range=(0.2, 0.8)) -> List[Job]:
    """A reproducible job mix: Poisson arrivals at `rate` jobs/s, n uniform
    over n_choices, p uniform in p_range, m log-uniform in m_range,
    h uniform in h_range (all draws from the counter-based generator)."""
    u = dg._unit(dg._column_keys(dg._stream_key(seed, dg.S_SERVE), np.arange(count)),
                 np.arange(6))
    jobs, t = [], 0.0
    for i in range(count):
        t += -math.log1p(-u[i, 0]) / rate
        n = int(n_choices[min(len(n_choices) - 1, int(u[i, 1] * len(n_choices)))])
        p = int(p_range[0] + min(p_range[1] - p_range[0], int(u[i, 2] * (p_range[1] - p_range[0] + 1))))
        m = int(round(math.exp(math.log(m_range[0]) + u[i, 3] * (math.log(m_range[1]) - math.log(m_range[0])))))
        h = float(h_range[0] + (h_range[1] - h_range[0]) * u[i, 4])
        jobs.append(Job(id=i, arrival=t, n=n, p=p, m=m, h=h, seed=seed + 1000 + i))
    return jobs


class Executor:
    """What the scheduler needs from a device."""

    def footprint(self, job: Job) -> int:
        raise NotImplementedError

    def admit(self, job: Job) -> None:
        """Factor M and whiten the fixed part; raise on failure."""
        raise NotImplementedError

    def submit_round(self, items: List[tuple]) -> object:
        """items: (job, snp0, nsnp); returns a token for poll/wait."""
        raise NotImplementedError

    def poll(self, token) -> bool:
        raise NotImplementedError

    def wait(self, token) -> None:
        raise NotImplementedError

    def release(self, job: Job) -> None:
        raise NotImplementedError


class Scheduler:
    """Admission by footprint, round composition, completion bookkeeping."""

    def __init__(self, executor: Executor, budget_bytes: int, max_items: int = 16,
                 inflight: int = 4, clock=time.monotonic, sleep=time.sleep,
                 target_cols: int = 32768, max_mult: int = 16, log=None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_items = max_items
        self.inflight = inflight
        self.clock = clock
        self.sleep = sleep
        # a round should give the device at least target_cols genotype
        # columns (32,768: one 128-column slab per compute unit, the widest
        # and, per column, fastest form of the solve); with few active jobs
        # every job's item grows by a common factor (up to max_mult), which
        # keeps the items of a round equal
        self.target_cols = target_cols
        self.max_mult = max_mult
        self.log = log
        self.used = 0
        self.peak_used = 0
        self.rounds = 0
        self.items = 0

    def run(self, jobs: List[Job]) -> Dict:
        jobs = sorted(jobs, key=lambda j: j.arrival)
        for j in jobs:
            j.block = j.block or job_block(j.n)
            j.max_block = j.max_block or min(max(j.block, 65536), j.block * self.max_mult)
        t0 = self.clock()
        arrived: List[Job] = []
        active: List[Job] = []
        queue: List[tuple] = []          # (token, items)
        nxt = 0
        rr = 0
        while True:
            now = self.clock() - t0
            while nxt < len(jobs) and jobs[nxt].arrival <= now:
                arrived.append(jobs[nxt])
                nxt += 1
            # admission in arrival order; a job larger than the whole budget fails
            while arrived:
                j = arrived[0]
                need = self.ex.footprint(j)
                if need > self.budget:
                    j.state, j.error = "failed", f"footprint {need} exceeds the budget {self.budget}"
                    arrived.pop(0)
                    continue
                if self.used + need > self.budget:
                    break
                arrived.pop(0)
                try:
                    self.ex.admit(j)
                except Exception as e:  # isolate the failure to this job
                    j.state, j.error = "failed", f"{type(e).__name__}: {e}"
                    j.finished = self.clock() - t0
                    if self.log:
                        self.log(f"t={j.finished:.2f}s job {j.id} failed at admission: {j.error}")
                    continue
                j.state, j.admitted = "active", self.clock() - t0
                j._need = need
                self.used += need
                self.peak_used = max(self.peak_used, self.used)
                active.append(j)
                if self.log:
                    self.log(f"t={j.admitted:.2f}s admit job {j.id} (n={j.n}, p={j.p}, m={j.m}), "
                             f"{len(active)} active, {self.used / 2**30:.1f} GiB used")
            # compose and queue a round
            if len(queue) < self.inflight:
                ready = [j for j in active if j.submitted < j.m]
                if ready:
                    items = []
                    k = len(ready)
                    pick = [ready[(rr + i) % k] for i in range(min(k, self.max_items))]
                    base = sum(j.block for j in pick)
                    mult = max(1, min(self.max_mult, -(-self.target_cols // base)))
                    # genotype bytes of a round are bounded by the executor's
                    # staging (a share per item, so that every picked job gets one)
                    cap = getattr(self.ex, "max_round_bytes", None)
                    for j in pick:
                        nsnp = min(j.block * mult, j.max_block, j.m - j.submitted)
                        if cap:
                            nsnp = max(1, min(nsnp, cap // len(pick) // j.n))
                        items.append((j, j.submitted, nsnp))
                        j.submitted += nsnp
                    rr = (rr + len(items)) % max(k, 1)
                    queue.append((self.ex.submit_round(items), items))
                    self.rounds += 1
                    self.items += len(items)
                    continue
            # retire finished rounds (in order)
            progressed = False
            while queue and (self.ex.poll(queue[0][0]) or len(queue) >= self.inflight):
                tok, items = queue.pop(0)
                self.ex.wait(tok)
                fin = self.clock() - t0
                for (j, s0, nsnp) in items:
                    j.completed += nsnp
                    if j.completed >= j.m and j.state == "active":
                        j.state, j.finished = "done", fin
                        self.ex.release(j)
                        self.used -= j._need
                        active.remove(j)
                        if self.log:
                            self.log(f"t={fin:.2f}s job {j.id} done, latency "
                                     f"{fin - j.arrival:.2f}s, {len(active)} active")
                progressed = True
            if progressed:
                continue
            if nxt >= len(jobs) and not arrived and not active and not queue:
                break
            if not queue and not [j for j in active if j.submitted < j.m]:
                # idle: wait for the next arrival (or for memory, which cannot
                # free up without active jobs)
                if nxt < len(jobs):
                    self.sleep(max(0.0, min(0.05, jobs[nxt].arrival - (self.clock() - t0))))
                elif arrived and not active:
                    for j in arrived:
                        j.state, j.error = "failed", "cannot be admitted"
                    arrived.clear()
            elif queue:
                self.sleep(0.0005)
        t_end = self.clock() - t0
        return summarize(jobs, t_end, self)


def summarize(jobs: List[Job], t_end: float, sched: Optional[Scheduler] = None) -> Dict:
    done = [j for j in jobs if j.state == "done"]
    lat = np.array([j.finished - j.arrival for j in done]) if done else np.array([np.nan])
    wait = np.array([j.admitted - j.arrival for j in done]) if done else np.array([np.nan])
    solved = sum(j.m for j in done)
    first = min(j.arrival for j in jobs) if jobs else 0.0
    flops = sum(float(j.n) ** 2 * j.m for j in done)
    out = {
        "jobs": len(jobs), "done": len(done), "failed": sum(j.state == "failed" for j in jobs),
        "makespan_s": t_end - first, "solves": solved,
        "solves_per_s": solved / max(t_end - first, 1e-9),
        "whitening_tflops": flops / max(t_end - first, 1e-9) / 1e12,
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(np.max(lat)), "admission_wait_p50_s": float(np.percentile(wait, 50)),
        "admission_wait_p99_s": float(np.percentile(wait, 99)),
    }
    if sched is not None:
        out.update({"rounds": sched.rounds, "items_per_round": sched.items / max(sched.rounds, 1),
                    "peak_footprint_bytes": sched.peak_used, "budget_bytes": sched.budget})
    return out


class GpuExecutor(Executor):
    """Jobs on the device through libgls.so.

    Per job: M = h*Phi_n + (1-h)*I + 1e-3*I built on the device from a
    resident Phi per cohort size (input construction), factored by
    gls_factor on the job's own stream, the fixed part whitened, one handle
    whose workspace holds one block, and the job's output b (m x p, on the
    device).  Genotypes: per round, the items' blocks are produced on the
    host into a pinned staging slot and copied to the slot's device buffer
    on a copy stream (`ingest="host"`, the default), or generated directly in
    device memory by the device twin of the generator (`ingest="device"`,
    no transfer).  Rounds run on one compute stream."""

    def __init__(self, precision: str = "fp64", phi: Optional[Dict[int, object]] = None,
                 keep_results: bool = False, ingest: str = "host",
                 slot_bytes: int = 1 << 30, streams: int = 2, slots: int = 5):
        import torch
        from . import gls
        self.torch, self.gls = torch, gls
        gls.lib()
        assert ingest in ("host", "device")
        self.ingest = ingest
        if ingest == "device":
            dg._dlib()
        self.precision = precision
        # rounds alternate over `streams` compute streams, so that the next
        # round's work-groups take the compute units the previous round's
        # last slabs leave free (no device-wide barrier between rounds); a
        # job keeps one handle (workspace) per stream
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.stream = self.streams[0]
        self.copy_stream = torch.cuda.Stream()
        self.phi = phi if phi is not None else {}
        self.state = {}
        self.keep_results = keep_results
        self.results = {}
        # (slack for the 256-byte alignment of each item in a slot)
        self.max_round_bytes = slot_bytes - (1 << 20) if ingest == "host" else None
        # staging slots: pinned host buffer, device buffer, and the events
        # that free them (copy done: pinned reusable; round done: device
        # buffer reusable)
        self.slots = []
        if ingest == "host":
            for _ in range(slots):
                self.slots.append({
                    "host": torch.empty(slot_bytes, dtype=torch.int8).pin_memory(),
                    "dev": torch.empty(slot_bytes, dtype=torch.int8, device="cuda"),
                    "copied": torch.cuda.Event(), "done": torch.cuda.Event()})
        self.round_no = 0
        self.ingest_host_s = 0.0    # host time producing genotypes
        self.ingest_bytes = 0
        # device timeline of the rounds: (start event, end event, whitening
        # flops, whether the previous round was still on the device when
        # this one was submitted)
        self.timeline = []

    def staging_bytes(self) -> int:
        """Device memory the executor holds besides the jobs' footprints."""
        return sum(int(sl["dev"].numel()) for sl in self.slots)

    def _phi(self, n: int):
        if n not in self.phi:
            w = dg.SERVE_BASE.replace(n=n, q=2 * n)
            self.phi[n] = self.torch.from_numpy(dg.make_phi(w)).cuda()
        return self.phi[n]

    def footprint(self, job: Job) -> int:
        p = self.gls.PRECISIONS[self.precision]
        blk = job.max_block or job.block or job_block(job.n)
        b = self.gls.gls_footprint_bytes(job.n, job.p_L, 1, 1, blk, p)
        # the workspaces of the handles forked for the other streams
        b += (len(self.streams) - 1) * (b - self.gls.gls_footprint_bytes(job.n, job.p_L, 1, 1, 0, p))
        if self.ingest == "device":
            b += job.n * blk                                   # genotype block
        b += job.m * job.p * 8 + job.m * 4                     # b and info
        b += job.n * job.n * 8                                 # M while factoring
        return int(b)

    def admit(self, job: Job) -> None:
        torch, gls = self.torch, self.gls
        w = job.workload()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            phi = self._phi(job.n)
            # column-major like phi (which is symmetric): no layout copy later
            M = torch.empty_strided(phi.shape, (1, phi.shape[0]), dtype=phi.dtype, device=phi.device)
            torch.mul(phi, job.h, out=M)
            M.diagonal().add_(1.0 - job.h + w.diag_shift)
            XL = torch.from_numpy(np.asfortranarray(dg.make_XL(w))).cuda()
            Y = torch.from_numpy(np.asfortranarray(dg.make_Y(w))).cuda()
        s.synchronize()
        c = gls.Cohort(M, precision=self.precision, stream=s)
        del M
        c.whiten_fixed(XL, Y, intercept_col=0)
        blk = job.max_block or job.block
        c.reserve(blk)
        hs = [c]
        for st in self.streams[1:]:
            f = c.fork(st)
            f.reserve(blk)
            hs.append(f)
        s.synchronize()
        xbuf = None
        if self.ingest == "device":
            xbuf = torch.empty((blk, job.n), dtype=torch.int8, device="cuda").t()
        B = torch.empty((job.m, 1, job.p), dtype=torch.float64, device="cuda")
        info = torch.empty((job.m,), dtype=torch.int32, device="cuda")
        self.state[job.id] = (hs, xbuf, B, info, w)

    def submit_round(self, items):
        torch, gls = self.torch, self.gls
        k = self.round_no % len(self.streams)
        stream = self.streams[k]
        sp = stream.cuda_stream
        works = []
        behind = bool(self.timeline) and not self.timeline[-1][1].query()
        if self.ingest == "device":
            for (job, s0, nsnp) in items:
                hs, xbuf, B, info, w = self.state[job.id]
                # one genotype buffer per job: its rounds stay on one stream
                stream, sp, k = self.streams[0], self.streams[0].cuda_stream, 0
                dg.make_XR_device(w, s0, nsnp, xbuf, sp)
                works.append(gls.gls_work(hs[k].h, nsnp, 1, xbuf.data_ptr(), job.n,
                                          B[s0:s0 + nsnp].data_ptr(), job.p,
                                          info[s0:s0 + nsnp].data_ptr()))
        else:
            slot = self.slots[self.round_no % len(self.slots)]
            # the pinned buffer is free once its previous copy has landed
            slot["copied"].synchronize()
            t0 = time.perf_counter()
            off, offs = 0, []
            for (job, s0, nsnp) in items:
                hs, xbuf, B, info, w = self.state[job.id]
                nb = job.n * nsnp
                assert off + nb <= slot["host"].numel(), "round exceeds the staging slot"
                view = slot["host"][off:off + nb].view(nsnp, job.n).numpy()
                dg.make_XR(w, s0, nsnp, out=view)          # the job's genotypes, on the host
                offs.append(off)
                off = (off + nb + 255) // 256 * 256
            self.ingest_host_s += time.perf_counter() - t0
            self.ingest_bytes += off
            # the device buffer is free once the round that used it has finished
            self.copy_stream.wait_event(slot["done"])
            with torch.cuda.stream(self.copy_stream):
                slot["dev"][:off].copy_(slot["host"][:off], non_blocking=True)
            slot["copied"].record(self.copy_stream)
            stream.wait_event(slot["copied"])
            base = slot["dev"].data_ptr()
            for (job, s0, nsnp), o in zip(items, offs):
                hs, xbuf, B, info, w = self.state[job.id]
                works.append(gls.gls_work(hs[k].h, nsnp, 1, base + o, job.n,
                                          B[s0:s0 + nsnp].data_ptr(), job.p,
                                          info[s0:s0 + nsnp].data_ptr()))
        t_start = torch.cuda.Event(enable_timing=True)
        t_start.record(stream)
        rc = gls.gls_solve_multi(works, sp)
        if rc != 0:
            raise gls.GLSError(rc, "gls_solve_multi")
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(stream)
        self.timeline.append((t_start, ev, sum(float(job.n) ** 2 * nsnp for (job, _, nsnp) in items),
                              behind))
        if self.ingest == "host":
            slot["done"].record(stream)
        self.round_no += 1
        return ev

    def timeline_summary(self) -> Dict:
        """Rounds as the device ran them.  device_busy_s: time with at least
        one round on the device (rounds on different streams may overlap;
        overlap_s is the time they did); round_whitening_tflops: whitening
        rate over that time; queued_gap_s: time between rounds when the next
        one had been submitted before the previous finished (launch and
        ingestion overhead, what a persistent launch could recover);
        idle_gap_s: time the device waited for arrivals."""
        for st in self.streams:
            st.synchronize()
        if not self.timeline:
            return {"rounds": 0}
        t0 = self.timeline[0][0]
        iv = sorted((t0.elapsed_time(a) * 1e-3, t0.elapsed_time(b) * 1e-3, w, behind)
                    for (a, b, w, behind) in self.timeline)
        busy = queued_gap = idle_gap = 0.0
        cur_s, cur_e = iv[0][0], iv[0][1]
        for (s0, e0, _, behind) in iv[1:]:
            if s0 > cur_e:
                if behind:
                    queued_gap += s0 - cur_e
                else:
                    idle_gap += s0 - cur_e
                busy += cur_e - cur_s
                cur_s, cur_e = s0, e0
            else:
                cur_e = max(cur_e, e0)
        busy += cur_e - cur_s
        work = sum(x[2] for x in iv)
        total = sum(x[1] - x[0] for x in iv)
        return {"rounds": len(iv), "streams": len(self.streams), "device_busy_s": busy,
                "round_whitening_tflops": work / max(busy, 1e-12) / 1e12,
                "overlap_s": total - busy, "queued_gap_s": queued_gap, "idle_gap_s": idle_gap,
                "queued_gap_frac_of_busy": queued_gap / max(busy, 1e-12),
                "ingest_host_s": self.ingest_host_s, "ingest_gb": self.ingest_bytes / 1e9,
                "ingest": self.ingest}

    def poll(self, token) -> bool:
        return token.query()

    def wait(self, token) -> None:
        token.synchronize()

    def release(self, job: Job) -> None:
        hs, xbuf, B, info, w = self.state.pop(job.id)
        if self.keep_results:
            self.results[job.id] = (B.cpu().numpy(), info.cpu().numpy())
        for h in hs[1:]:
            h.free()
        hs[0].free()
