"""FP64 CPU oracle for the energy-coupled neutrino-matter interaction rates.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call, link or run this
package: only the test suite, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code, tables or constants generator with the HIP library; both sides only
read the same seeded inputs (``paper_1404_1719_amd.synth``).

The paper (Marek et al., "Towards Petaflops Capability of the VERTEX Supernova Code")
names the emission, absorption and scattering rates of neutrinos as one component of the
model (Sect. 2.1, list of components) and gives no formula for them. The kernel definition
implemented here is the standard massless-electron V-A one, written out step by step:

* ``physics``   constants and species couplings;
* ``angular``   angular weights H (phi-averaged |M|^2 integrated over the momentum transfer),
                evaluated by exact term-by-term antiderivatives of a Laurent polynomial in k;
* ``rule``      the quadrature rule R over the electron energy (node placement);
* ``rates``     kernel quadrature, detailed-balance completion, species combination and the
                contraction with f into eta, chi (the paper's J/H moment interface, Eq. 1);
* ``grad``      reverse-mode products by complex-step differentiation of ``rates``;
* ``converged`` adaptive (scipy) integrals that measure the rule's own discretisation error.

Parity status of each function is stated in its module header.
"""
