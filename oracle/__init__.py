"""Plain, slow, FP64 CPU oracle of the N-component free-energy lattice Boltzmann
update (Rennick, Zhang, Bingert, Krause, Kusumaatmaja, arXiv 2605.22214).

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
The HIP library never calls, links or reads anything here, and nothing here
imports the HIP library: the two share no code, headers, tables or helpers.

Modules
-------
lattice   D2Q9 (Sec. III) and D3Q19 (the textbook set the paper points to).
coeffs    alpha, gamma (Eqs. alpha1/alpha2), Lambda (Eq. ngamma), Theta
          (the Theta system below Eq. P), and the factored tables.
potential chemical potentials and the flux potential mu~_i in the literal form
          of Eq. MU and in the factored form.
step      one vectorised time step (Sec. III A-C) over the whole lattice.
naive     the same step written node by node in pure Python (tiny lattices).
diag      FP64 invariants: mass, momentum, max|C|, sum-rule deviation.
analysis  closed forms used as pins: Neumann angles (Eq. neucosine), layered
          Poiseuille (Eqs. piecewisequad, velocityprof), Laplace law, linear
          dispersion of the Cahn-Hilliard LBE.
"""
