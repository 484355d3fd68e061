"""ConstructMicroBatch oracle -- TEST INFRASTRUCTURE ONLY.

Algorithm 1 of the paper (Sec. III-C) in its own notation, with the metrics
of Eq. 4-6:

* Buff_(i,j): how long dataset j of the temporary micro-batch i has waited
  (now - its creation time); Part_(i,j): its rows;
* AvgThPut_(i-1) = rows of the completed batches / their processing time (Eq. 4);
* EstMaxLat_i = max_j Buff_(i,j) + sum_j Part_(i,j) / AvgThPut_(i-1) (Eq. 6);
* MaxLat_k = max_j Buff_(k,j) + Proc_k of a completed batch (Eq. 5);
* SlideTime > 0 (sliding window): admit when EstMaxLat_i >= SlideTime;
  SlideTime = 0 (tumbling window): admit when EstMaxLat_i >= the mean of the
  past MaxLat (Eq. 3).

Readings where the paper leaves a gap: the mean of Eq. 3 is over the batches
completed so far; the first batch is admitted as soon as it is non-empty and
the processing term of Eq. 6 is left out until one batch has completed
(AvgThPut is undefined before); one poll period is added to the estimate
(admission happens at the first poll that would otherwise overshoot); an
explicit deadline can replace SlideTime for queries without a window; with
``poll_idle`` the admission test also runs on polls that bring no new data.
"""
from __future__ import annotations


class ConstructMicroBatch:
    def __init__(self, slide_ms=0.0, deadline_ms=0.0, poll_ms=10.0, poll_idle=True):
        self.slide_time = slide_ms
        self.deadline = deadline_ms
        self.poll = poll_ms
        self.poll_idle = poll_idle
        self.buffered_files = []  # (creation time, rows)
        self.done = []            # (rows, Proc, MaxLat) of completed batches
        self.admitted = 0

    def avg_thput(self):
        rows = sum(r for r, _, _ in self.done)
        proc = sum(p for _, p, _ in self.done)
        return rows / proc if proc > 0 else None

    def est_max_lat(self, now, tmp):
        buff = max(now - c for c, _ in tmp)
        thput = self.avg_thput()
        part = sum(r for _, r in tmp)
        return buff + (part / thput if thput else 0.0)

    def target(self):
        if self.deadline > 0:
            return self.deadline
        if self.slide_time > 0:
            return self.slide_time
        if self.done:
            return sum(m for _, _, m in self.done) / len(self.done)
        return 0.0

    def poll_once(self, now, new_files):
        """Returns (admitted, micro-batch) with micro-batch a list of (creation time, rows)."""
        if not new_files and not (self.poll_idle and self.buffered_files):
            return False, []
        tmp = self.buffered_files + sorted(new_files, key=lambda f: f[0])
        if not tmp:
            return False, []
        est = self.est_max_lat(now, tmp)
        if self.admitted == 0 or est + self.poll >= self.target():
            self.buffered_files = []
            self.admitted += 1
            return True, tmp
        self.buffered_files = tmp
        return False, []

    def complete(self, rows, proc, max_lat):
        self.done.append((rows, proc, max_lat))


def fixed_trigger_batches(trigger_ms, arrivals, proc_of, t_end):
    """The default micro-batch model the paper starts from (Sec. II-B, Fig. 4(a)):
    a batch is cut every trigger interval and holds every dataset that arrived
    since the last cut; when processing overruns the interval, the next cut
    waits for it to finish (the interval stretches).  One executor.
    Returns [(cut time, datasets, MaxLat)] with MaxLat as in Eq. 5."""
    out, nxt, t = [], 0, float(trigger_ms)
    while t <= t_end:
        batch = []
        while nxt < len(arrivals) and arrivals[nxt] <= t:
            batch.append(arrivals[nxt])
            nxt += 1
        if batch:
            proc = proc_of(len(batch))
            out.append((t, len(batch), (t - min(batch)) + proc))
            t = max(t + trigger_ms, t + proc)
        else:
            t += trigger_ms
    return out
