"""Plain, slow FP64 CPU oracle of the nuance transit search (arXiv:2402.06835).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call anything here.
The product path (the HIP library and its Python binding) never does, and
this package never imports the product path: the two share no code.

Contents (each function cites the passage it follows):

* ``oracle.gp``        SHO covariance (Appendix A), K = k + sigma_w^2 I, Cholesky,
                       log-determinant.
* ``oracle.linear``    The linear search (Section 2.2): per (epoch, duration)
                       cell, the full generalised-least-squares fit of
                       Eq. 6 with X = [trend | box] and the log-likelihood
                       of Eq. 5, reported as depth, depth variance and the
                       log-likelihood gain over the trend-only fit.
* ``oracle.periodic``  The periodic search (Section 2.3-2.4): interpolation of
                       the linear-search grid onto phases, the common-depth
                       combination of Eq. 8 with the estimates of Eq. B4,
                       the argmax of Eq. 9 and Q(P) = depth/sigma.
* ``oracle.segments``  The periodic search over several segments (sectors), each
                       with its own linear search, on one global lattice.
* ``oracle.templates`` The single-event search with a non-box base model in
                       the last column (Section 4.4, prospects: limb-darkened
                       transits, exocomets): the same fit with a shape per
                       duration in place of the box.
* ``oracle.multiplanet`` The iterative search for several candidates (Section 3.3):
                       mask the found candidate's transit windows in the
                       linear-search products and search again.
* ``oracle.learned``   The hyperparameter fit the search needs first (Section
                       3.2: maximum likelihood with the trend solved
                       linearly) and the learned warm start for it: the
                       counter-based random numbers and GP sampler of the
                       training data, the CNN input, the network with its
                       gradient and Adam, the trend-profiled likelihood by
                       dense Cholesky and by Kalman filter, the plain
                       Lomb-Scargle start and BFGS.

Readings of passages where the paper is silent or inconsistent are listed
in each module header. Parity unpinned (no worked numbers in the paper):
the sign of the log-ratio term of Eq. 8 (both signs are implemented), the
box-edge convention, linear interpolation in the lattice index, and the
tie rule of the argmax.
"""
