"""CPU FP64 oracle for the stochastic Kraus-trajectory noise method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU product
path (``paper_2210_15874_amd``) never imports, links or runs anything here, and
this package imports nothing from it: the two share only the seeded inputs of
``workloads``.

What it computes (all complex128 / float64, plain and slow on purpose):

* ``density``      exact density-matrix evolution: every gate as U rho U^dagger,
                   every channel as the operator sum of Eq.(1) (Sec. III-F).
* ``trajectories`` the stochastic ensemble estimator of Sec. III-G: gate by gate,
                   and after each gate, for each of its channels, one uniform
                   draw picks a Kraus operator which is inserted literally
                   (normalised by the square root of its selection probability);
                   the resulting statevectors are averaged to rho_hat, its
                   diagonal (sigma_approx) and the MaxCut energy <C>.
* ``philox``       Philox4x32-10 (Salmon et al., SC'11), the counter-based draw.
* ``channels``     Kraus sets (Sec. III-F), selection probabilities and the
                   integer thresholds that turn a 32-bit draw into an index.
* ``metrics``      Eq.(2) error, Uhlmann fidelity, trace distance, Frobenius.
* ``sampling``     bitstrings drawn from sigma_approx by inverse-transform
                   sampling of its running sums.

Pins (tests/test_oracle_*.py, run with ``-m "not gpu"``): channel closed forms,
trace/Hermitian/PSD invariants, the noiseless limit against the p=1 QAOA
closed form of Wang et al., exhaustive outcome enumeration against the exact
density matrix, the convergence law of the estimator, Philox against the
independent rocRAND implementation, and the bitstring sampler against
hand-computed samples, stratified counts and a chi-square bound.  Parity unpinned: <C> with noise at sizes
where no exact density matrix fits (n > 12); there only same-draw comparison and
the stated standard error apply.
"""
