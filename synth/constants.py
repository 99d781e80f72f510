"""Physical constants (CODATA 2018 / SI exact values).

The paper gives no constants of its own; these are the standard values for
the quantities its setup section names (electron and argon masses, the
elementary charge, Boltzmann's constant, the torr).
"""

QE = 1.602176634e-19        # elementary charge [C] (exact, SI 2019)
KB = 1.380649e-23           # Boltzmann constant [J/K] (exact, SI 2019)
ME = 9.1093837015e-31       # electron mass [kg] (CODATA 2018)
AMU = 1.66053906660e-27     # atomic mass unit [kg] (CODATA 2018)
M_AR = 39.948 * AMU         # argon atom / Ar+ ion mass [kg]
EPS0 = 8.8541878128e-12     # vacuum permittivity [F/m] (CODATA 2018)
TORR = 101325.0 / 760.0     # 1 Torr in Pa (exact by definition)


def gas_density(p_torr, T_gas=300.0):
    """Neutral number density n_g = p / (k_B T) in m^-3 for p given in Torr."""
    return p_torr * TORR / (KB * T_gas)
