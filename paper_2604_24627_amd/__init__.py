"""axpic -- MI355X-native Monte-Carlo axion operators for particle-in-cell plasmas.

Importing the package loads nothing; ``paper_2604_24627_amd.axpic.load()``
binds libaxpic.so (HIP, gfx950) and ``paper_2604_24627_amd.sim.AxpicSim``
drives whole time steps.  ``paper_2604_24627_amd.inputs`` builds the seeded
synthetic plasmas.
"""
__all__ = ["axpic", "sim", "inputs", "build"]
