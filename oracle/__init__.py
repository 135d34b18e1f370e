"""FP64 CPU oracle of the mass-spring method -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy implementation of what the simulator computes, written
from the paper (Clay et al., "A Massively-Parallel 3D Simulator for Soft and Hybrid Robots"):

* ``lattice``     voxel lattice -> masses and springs (section "Generating a Lattice")
* ``layout``      space-filling-curve renumbering and per-mass incidence lists (the duplicated
                  mass->spring connectivity of section "GPU Implementation")
* ``physics``     eq. (2) forces, actuated rest lengths, contact plane with friction,
                  semi-implicit (symplectic) Euler in the form of eqs. (3)-(4), damping
* ``diagnostics`` energies of section "Energy Conservation Tests", momentum, centre of mass
* ``adjoint``     reverse-mode derivative of the discrete step (gait gradients)
* ``mlp``         FP64 multilayer perceptron used to check the surrogate kernels

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  It shares no code with the native library and never imports it.
Functions whose result has no independent pin say "parity unpinned" in their docstring.
"""
