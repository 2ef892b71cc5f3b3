"""Plain FP64 CPU oracle for the COLA particle-mesh method (Izard, Crocce & Fosalba,
ICE-COLA, arXiv:1509.04685).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or calls this
package; only the test suite, the smoke check and the CPU-baseline leg of the benchmark
do.  It shares no code with the HIP path: every step is written out here, in float64,
in the order the method defines it, so that a reader can check it against the paper.

Modules
-------
cosmology  background expansion, linear growth D1, second-order growth D2, the kick and
           drift time integrals, the time nodes of Eq. 3, the BBKS linear spectrum.
noise      Philox4x64-10 counter-based generator and Box-Muller white noise.
lpt        Gaussian field and the first/second-order Lagrangian displacements.
pm         cloud-in-cell assignment, the Poisson/gradient solve, CIC interpolation.
cola       the COLA kick-drift-kick integrator in the frame comoving with 2LPT.
power      the matter power-spectrum estimator.
learned    the coarse-mesh force-correction network: forward, backward, particle loss.
fof        friends-of-friends groups, the halo catalogue and the binned Warren mass function.
"""

from . import cosmology, noise, lpt, pm, cola, power, learned, fof  # noqa: F401
